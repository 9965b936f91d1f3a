/*
 * discomatch.h -- C ABI of the MI355X (gfx950) dual solver for the
 * geometrically consistent product-triangle ILP of DiscoMatch
 * (arXiv 2310.08230).
 *
 * The problem (Sec. 3.1, Eq. (P)):  min c^T x  s.t.  A x = b,  x in {0,1}^|P|,
 * where P is the product space of triangle-triangle, triangle-edge and
 * triangle-vertex matching elements, A stacks the closedness rows
 * (A^d x = 0) and the projection rows of both shapes (A^M x = 1, A^N x = 1),
 * and c is built from per-vertex descriptors and mixed areas (Sec. 4.2,
 * Eq. (cost)).  The solver works on its Lagrangean decomposition dual
 * (Sec. 3.2, Eq. (D)): one subproblem per row, multipliers lambda^j_i with
 * sum_{j in J_i} lambda^j_i = c_i.
 *
 * Conventions for every entry point:
 *  - Pointers marked [device] are device memory of the context's GPU, owned by
 *    the caller, read or written on the context's stream in stream order.
 *    Pointers marked [host] are host memory owned by the caller.
 *  - Functions that return host values (sizes, bounds, flags) synchronise the
 *    context's stream before returning; the others only enqueue work.
 *  - Nothing throws or exits.  A negative return is an error; its message is
 *    in dm_last_error(ctx).  A context is not thread-safe; use one per stream.
 *  - The context owns the product space, the incidence and the solver state
 *    it builds (device memory it allocates itself, released by dm_destroy).
 */
#ifndef DISCOMATCH_H
#define DISCOMATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dm_status;

enum {
  DM_OK = 0,
  DM_ERR_INVALID_ARG = -1, /* bad pointer, size, index or order of calls     */
  DM_ERR_MESH = -2,        /* not a closed, oriented 2-manifold             */
  DM_ERR_GENUS = -3,       /* Euler characteristics of X and Y differ       */
  DM_ERR_INFEASIBLE = -4,  /* A x = b has no 0/1 solution (proved by presolve) */
  DM_ERR_NONFINITE = -5,   /* NaN or Inf in vertices or descriptors         */
  DM_ERR_WORKSPACE = -6,   /* a size exceeds what the kernels support       */
  DM_ERR_HIP = -7,         /* HIP runtime error                             */
  DM_ERR_STATE = -8        /* a prerequisite step has not been run          */
};

enum { DM_PREC_FP64 = 0, DM_PREC_FP32 = 1, DM_PREC_BF16 = 2 };

typedef struct dm_ctx dm_ctx;

/* A triangle mesh (Table "notation": V in R^{|V| x 3}, T in N^{|T| x 3}).
 * verts [device] float32 [nv*3]; faces [device] int32 [nf*3], counter-
 * clockwise seen from outside. */
typedef struct {
  int32_t nv, nf;
  const float* verts;
  const int32_t* faces;
} dm_mesh;

/* Sizes of a built product space (all counts after K-candidate pruning). */
typedef struct {
  int64_t n_prod_tri;  /* |P|: kept product triangles                       */
  int64_t n_rows_full; /* rows of A before presolve                         */
  int64_t nnz_full;    /* nonzeros of A before presolve                     */
  int64_t n_closed_full; /* closedness rows before presolve                 */
  int64_t n_free;      /* variables left free by presolve                   */
  int64_t n_fixed1;    /* variables presolve fixed to 1                     */
  int64_t n_rows;      /* rows of the presolved problem (the subproblems)   */
  int64_t nnz;         /* its nonzeros = number of multipliers lambda^j_i   */
  int64_t n_short_rows;/* closedness rows in the presolved problem          */
  int64_t n_edges_x, n_edges_y;
  int64_t n_cand;      /* |C|: candidate vertex pairs                       */
  int32_t presolve_rounds;
  int32_t max_short_row;
} dm_space_info;

/* Create a context on HIP device `device`; work is enqueued on `hip_stream`
 * (a hipStream_t, may be NULL for the default stream).  The memory the
 * library allocates itself (the build steps' arrays and temporaries, and the
 * solver state unless the caller supplies it with dm_set_workspace) comes
 * stream-ordered, on that stream, from a memory pool that the context creates
 * for itself and destroys in dm_destroy; the pool keeps freed blocks for the
 * context's later calls and leaves the device's default pool untouched.  The
 * context also keeps up to 4 GiB of the blocks it frees, by size, and hands
 * them to its later allocations of the same size without a runtime call
 * (dm_set_stream to another stream, an allocation that finds the pool out of
 * memory, and dm_destroy return them to the pool).  The stream must stay
 * valid until dm_destroy.  Errors: DM_ERR_INVALID_ARG (no
 * such device), DM_ERR_HIP (the pool or pinned host slots could not be
 * created). */
dm_status dm_create(int32_t device, void* hip_stream, dm_ctx** out);
/* Destroys ctx: synchronises its stream, frees what the library allocated
 * and destroys the context's pool; caller workspaces are not touched. */
dm_status dm_destroy(dm_ctx* ctx);
/* Message of the last error on ctx (empty string if none); owned by ctx. */
const char* dm_last_error(const dm_ctx* ctx);
/* Rebind the stream used by later calls; when it changes, the previous
 * stream is synchronised first. */
dm_status dm_set_stream(dm_ctx* ctx, void* hip_stream);

/* Caller-owned solver state (the "Ownership" of the C ABI: device buffers
 * may come from the caller, e.g. PyTorch tensors).  After a problem is built
 * (dm_build_product_space or dm_build_ilp, and after dm_fix_variables) the
 * Jacobi solver's state of one message precision has a known size:
 * dm_workspace_query gives it for stage DM_WS_SOLVE_FP32 or DM_WS_SOLVE_FP64
 * (two multiplier record buffers of n_free x 8 reals and the per-block bound
 * partials of a sweep).  dm_set_workspace hands the library a device buffer
 * of at least that many bytes, 256-byte aligned: from then on dm_dual_solve,
 * dm_lbfgs_solve and the sweeps of that precision keep their records and
 * partials there instead of allocating them.  The caller owns the buffer,
 * keeps it alive while it is attached and does not touch it between calls;
 * the library reads and writes it only on the context's stream.  ptr = NULL
 * detaches (the library allocates again).  A later problem may need more:
 * the solver calls then return DM_ERR_WORKSPACE until a larger buffer is
 * attached.  Errors: DM_ERR_INVALID_ARG (unknown stage, misaligned buffer),
 * DM_ERR_STATE (no problem built), DM_ERR_WORKSPACE (buffer too small).
 * Neither call synchronises. */
enum { DM_WS_SOLVE_FP32 = 0, DM_WS_SOLVE_FP64 = 1 };
dm_status dm_workspace_query(const dm_ctx* ctx, int32_t stage, size_t* bytes);
dm_status dm_set_workspace(dm_ctx* ctx, int32_t stage, void* ptr, size_t bytes);

/* Candidate vertex pairs (A2).  Distances d(m,n) = ||F_X(m) - F_Y(n)||_2 from
 * a tiled GEMM (prec = DM_PREC_BF16: BF16 MFMA on descriptors rounded to BF16
 * with FP32 accumulation; DM_PREC_FP32: FP32), then for every vertex of X the
 * K nearest vertices of Y by (d, index), and the converse.  The paper prunes
 * its product spaces only in the coarse-to-fine scheme (Sec. 5.2); the rule
 * here is the library's.
 *  FX [device] float32 [nvx*D] row-major; FY [device] float32 [nvy*D];
 *  cand_xy [device] int32 [nvx*K] out; cand_yx [device] int32 [nvy*K] out.
 *  The K nearest are selected exactly at any size (a radix selection of
 *  the (distance, index) keys for K <= 2048, a full sort otherwise).
 *  Errors: K < 1, K > nvx or nvy, K > 2048 when nvx or nvy exceeds 4096,
 *  nvx or nvy > 2^21, D < 1. */
dm_status dm_knn_candidates(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY,
                            int32_t nvy, int32_t D, int32_t K, int32_t prec, int32_t* cand_xy,
                            int32_t* cand_yx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as dm_knn_candidates, with the temporaries (an
 * error word, the squared distances and the BF16 operand copies) in a fixed
 * scratch array of 16 MiB that every GPU the library runs on holds until the
 * process ends.  No call allocates or frees memory.  Arguments, layouts and
 * errors as dm_knn_candidates; in addition DM_ERR_WORKSPACE when the
 * temporaries exceed 16 MiB: 4*nvx*nvy bytes of distances, plus
 * 2*D16*(nvx64 + nvy64) + 4*(nvx64 + nvy64) in BF16, with D16 = D rounded up
 * to 16 and nvx64, nvy64 rounded up to 64, each piece rounded up to 256 bytes
 * (about 2000 x 2000 vertices at D = 128).  Every call on one GPU shares
 * that GPU's array and leaves its last contents there; calls that overlap on
 * one GPU (other threads, other streams, other contexts) race and must be
 * serialised by the caller.  Synchronises (the finiteness check). */
dm_status dm_knn_candidates_noalloc(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY,
                                    int32_t nvy, int32_t D, int32_t K, int32_t prec, int32_t* cand_xy,
                                    int32_t* cand_yx);

/* Generic 0-1 ILPs (Appendix "Other ILPs": the solver is not specific to
 * matching): min c^T x subject to A x = b, x in {0,1}^n, every coefficient
 * +1 or -1, every variable in 1 to 5 rows, no variable twice in one row.
 * Rows with all coefficients +1 and b = 1 are exactly-one rows of any
 * length; the others have at most 64 entries.  The decomposition is that of
 * Eq. (D): one subproblem per input row and nothing else, so a variable in d
 * rows has d multipliers summing to its cost.  The full row order is
 * [other input rows | exactly-one input rows], each group in input order.
 * Presolve and the reduced problem follow as for the matching ILP, and every
 * solver entry point applies (multipliers, dual and quasi-Newton solves,
 * bounds, rounding, fixing, exact search); the ones that need meshes,
 * candidates or descriptor costs return DM_ERR_STATE.  Costs come from
 * dm_set_costs.
 *  row_ptr [device] int32 [n_rows + 1], starting at 0 and never decreasing,
 *  nnz = row_ptr[n_rows]; cols [device] int32 [nnz]; coefs [device] int8
 *  [nnz]; b [device] int32 [n_rows]; *info [host] out.
 *  Errors: DM_ERR_INVALID_ARG for malformed row pointers, a column out of
 *  range, a coefficient other than +-1, a variable in no row or in more
 *  than 5, or a variable twice in one row; DM_ERR_WORKSPACE for a row that
 *  is not exactly-one with more than 64 entries; DM_ERR_INFEASIBLE when
 *  presolve proves A x = b has no 0-1 solution.  Synchronises. */
dm_status dm_build_ilp(dm_ctx* ctx, int32_t n_vars, int32_t n_rows, const int32_t* row_ptr, const int32_t* cols,
                       const int8_t* coefs, const int32_t* b, dm_space_info* info);

/* Costs c [device] float64 [n_prod_tri] of the current problem (generic or
 * matching), replacing any built ones; the offset of the variables fixed to
 * 1 follows.  After it, dm_smoothed_backward (which differentiates the
 * descriptor costs) is refused until dm_build_costs runs again.
 * Errors: a non-finite cost.  Synchronises. */
dm_status dm_set_costs(dm_ctx* ctx, const double* cost);

/* Coarse-to-fine pruning (Sec. 5.2): a vertex matching found at a coarser
 * resolution restricts the candidate pairs at the next finer one to the
 * ring neighbourhoods of the matched vertices.  Three steps:
 *
 * dm_nearest_vertices: for each of the n points P (a coarse vertex's rest
 * position) the index of the nearest of the m points Q (fine vertices):
 * squared distances in FP64 (exact for FP32 coordinates), ties to the lower
 * index.  P [device] float32 [n*3], Q [device] float32 [m*3], out [device]
 * int32 [n].  Enqueue only. */
dm_status dm_nearest_vertices(dm_ctx* ctx, const float* P, int32_t n, const float* Q, int32_t m, int32_t* out);

/* dm_matched_pairs: the vertex pairs (m, n) that the selected elements of a
 * primal x use (the corners of the product triangles with x = 1), in
 * ascending order of m * nvY + n, on the context's product space.
 *  x [device] uint8 [n_prod_tri]; pairs [device] int32 [cap*2] out (m, n);
 *  *n_pairs [host] out (also when it exceeds cap, which is an error).
 *  Synchronises. */
dm_status dm_matched_pairs(dm_ctx* ctx, const uint8_t* x, int32_t* pairs, int32_t cap, int32_t* n_pairs);

/* dm_ring_candidates: for each seed pair (a, b) of fine vertices (a coarse
 * match placed on the fine meshes), every pair (u, v) with u in the ring
 * neighbourhood of a on X and v in that of b on Y (rings = 1: the vertex and
 * its neighbours; 2: also theirs) becomes a candidate; the union over the
 * seeds is returned as per-vertex lists in ascending order, both ways,
 * padded to the common length K by repeating the last entry (the layout of
 * dm_knn_candidates; dm_build_product_space ignores the repeats).
 *  Xf, Yf: the fine meshes (as for dm_build_product_space); seeds [device]
 *  int32 [n_seeds*2]; cand_xy [device] int32 [nvX*kcap] out, cand_yx
 *  [device] int32 [nvY*kcap] out (the first nv*K entries are used); *K
 *  [host] out.  Errors: a seed out of range, a ring over 512 members, K >
 *  kcap (DM_ERR_WORKSPACE, *K set), a fine vertex left without candidates
 *  (DM_ERR_INFEASIBLE).  Synchronises. */
dm_status dm_ring_candidates(dm_ctx* ctx, const dm_mesh* Xf, const dm_mesh* Yf, const int32_t* seeds,
                             int32_t n_seeds, int32_t rings, int32_t kcap, int32_t* cand_xy, int32_t* cand_yx,
                             int32_t* K);

/* Product space, constraints and presolve (A1, A3; Sec. 3.1, Eq. (P)).
 * Validates both meshes, enumerates every product triangle whose three
 * product vertices (m, n) lie in the candidate set C (the union of cand_xy and
 * cand_yx), builds the rows of A (closedness rows per undirected product edge
 * sorted by key, then one projection row per face of X, then per face of Y)
 * and runs integer unit propagation to a fixpoint.  Replaces any previous
 * space on ctx.  Synchronises; fills *info.
 *  X, Y [host] descriptors of device meshes; cand_* [device] as above.
 *  Errors: DM_ERR_MESH, DM_ERR_GENUS, DM_ERR_INFEASIBLE, DM_ERR_WORKSPACE. */
dm_status dm_build_product_space(dm_ctx* ctx, const dm_mesh* X, const dm_mesh* Y,
                                 const int32_t* cand_xy, const int32_t* cand_yx, int32_t K,
                                 dm_space_info* info);

/* Export arrays of the built space (for checks) into caller buffers [device]:
 *  DM_ARR_PV      int32 [n_prod_tri*3]  product-vertex ids m*nvy+n per corner
 *  DM_ARR_CODE    int32 [n_prod_tri*4]  (x class, x id, y class*8+pattern, y id),
 *                 class 0 face, 1 edge, 2 vertex
 *  DM_ARR_STATE   int8  [n_prod_tri]    -1 free, 0 or 1 fixed by presolve
 *  DM_ARR_ROW_KEY int64 [n_rows_full]   closedness: min*NPV+max (NPV = nvx*nvy);
 *                                       projection rows: face id
 *  DM_ARR_ROW_PTR int64 [n_rows_full+1], DM_ARR_ENT_VAR int64 [nnz_full],
 *  DM_ARR_ENT_COEF int32 [nnz_full], DM_ARR_ROW_B int32 [n_rows_full]
 *  DM_ARR_FREE_VAR int64 [n_free]       element of each free variable
 *  DM_ARR_RROW_ORIG int64 [n_rows], DM_ARR_RROW_PTR int64 [n_rows+1],
 *  DM_ARR_RENT_VAR int64 [nnz], DM_ARR_RENT_COEF int32 [nnz], DM_ARR_RROW_B int32 [n_rows]
 *  DM_ARR_EDGES_X / _Y int32 [n_edges*2] sorted (min, max) vertex pairs
 *  DM_ARR_CAND    uint8 [nvx*nvy]        1 where (m, n) is in C
 * dst [device] receives the array (enqueued only); it may be NULL when the
 * array is empty (e.g. the reduced rows of a problem presolve decided). */
enum {
  DM_ARR_PV = 0, DM_ARR_CODE, DM_ARR_STATE, DM_ARR_ROW_KEY, DM_ARR_ROW_PTR, DM_ARR_ENT_VAR,
  DM_ARR_ENT_COEF, DM_ARR_ROW_B, DM_ARR_FREE_VAR, DM_ARR_RROW_ORIG, DM_ARR_RROW_PTR,
  DM_ARR_RENT_VAR, DM_ARR_RENT_COEF, DM_ARR_RROW_B, DM_ARR_EDGES_X, DM_ARR_EDGES_Y, DM_ARR_CAND
};
dm_status dm_get_space(dm_ctx* ctx, int32_t which, void* dst);

/* Costs, Eq. (cost) (A4; Sec. 4.2): c_p = sum over the three product vertices
 * (m_v, n_v) of p of (A_X(m_v) + A_Y(n_v)) * d(m_v, n_v), with mixed vertex
 * areas (Meyer et al. 2003) of the posed meshes and the Euclidean descriptor
 * distance d, computed in FP64 (DM_PREC_FP64), FP32 (DM_PREC_FP32) or from a
 * BF16 MFMA GEMM with FP32 accumulation (DM_PREC_BF16).  Also sets the
 * solver's costs (stored in the message precision chosen later) and the
 * constant from variables fixed to 1.
 *  FX, FY [device] float32 as in dm_knn_candidates (same nvx, nvy as the space).
 *  cost [device] float32 [n_prod_tri] out, or NULL. */
dm_status dm_build_costs(dm_ctx* ctx, const float* FX, const float* FY, int32_t D, int32_t prec,
                         float* cost);

/* Initial multipliers lambda^j_i = c_i / |J_i| (A5; feasible for Eq. (D)).
 *  lambda [device] float32 or float64 (per msg_prec) [nnz], CSR order of the
 *  presolved rows (DM_ARR_RROW_PTR). */
dm_status dm_init_lambda(dm_ctx* ctx, int32_t msg_prec, void* lambda);

/* Jacobi min-marginal averaging (A6-A8; Sec. 3.2, the MMA step of Alg. 1):
 * per iteration every row computes its minimum and its min-marginal
 * differences M^j_i at the current lambda, the bound offset + sum of row
 * minima goes to lb_trace[t] (FP64, fixed summation order), and
 *   lambda^j_i <- lambda^j_i - omega * (M^j_i - mean_{k in J_i} M^k_i).
 * temperature > 0 replaces every min by the soft-min -T log sum exp(-./T)
 * (smoothed dual).  lambda is updated in place and must satisfy
 * sum_j lambda^j_i = c_i on entry (e.g. from dm_init_lambda).
 *  msg_prec DM_PREC_FP32 (lambda float32) or DM_PREC_FP64 (float64).
 *  lb_trace [device] double [iters] out, or NULL.  Enqueue only. */
dm_status dm_dual_solve(dm_ctx* ctx, int32_t iters, double omega, double temperature,
                        int32_t msg_prec, void* lambda, double* lb_trace);

/* Quasi-Newton powered MMA (Sec. 4.1, Alg. 1; Appendix "Quasi-Newton
 * Updates").  One iteration: the subgradient g (every row's minimising
 * assignment, 1 / 0 per multiplier); the direction d^ = H g by the L-BFGS
 * two-loop recursion over the last `history` accepted pairs (H = I without
 * history, H0 = (s^T y / y^T y) I of the newest pair otherwise); d = d^ minus
 * its mean over each variable's rows (keeps sum_j lambda^j_i = c_i);
 * FindStepSize: from the previous step size, up to max_search rescalings by
 * step_up (the trial did not lose against E(lambda)) or step_down (it did),
 * stopping once a trial gains Delta_min = 1e-6 (E(lambda^1) - E(lambda^0))
 * (no early stop in the first iteration), keeping the best trial; the step
 * lambda += gamma d only when that trial beats E(lambda); one Jacobi MMA
 * iteration with omega; then the pair s = lambda_new - lambda_old,
 * y = g_old - g_new joins the history when s^T y >= eps (L-BFGS acting on -E).
 * Dots are summed in FP64 in a fixed order.
 * resume != 0 continues the search state of the previous call on this
 * context (history pairs, step size, Delta_min) from the given lambda; it
 * needs an earlier call with the same msg_prec and history on the same costs
 * (DM_ERR_STATE otherwise).  resume = 0 starts afresh.
 *  lambda [device] float32 / float64 (msg_prec) [nnz] in/out, feasible on entry.
 *  lb_trace [device] double [iters + 1] out or NULL: E at the start of every
 *  iteration and at the end.  gamma_trace [device] double [iters] out or NULL:
 *  the step size FindStepSize returned.  taken [device] int32 [iters] out or
 *  NULL: 1 where the quasi-Newton step was applied.  The context keeps the
 *  work buffers (history + 1 s and y vectors) until it is destroyed; reads
 *  one flag back to the host per iteration (synchronises). */
typedef struct {
  int32_t history;      /* m, number of stored (s, y) pairs, >= 0 */
  int32_t max_search;   /* K, rescalings per FindStepSize, >= 1 */
  double omega;         /* MMA damping, (0, 1] */
  double eps;           /* curvature threshold */
  double step_up;       /* > 1 */
  double step_down;     /* in (0, 1) */
  double gamma0;        /* first step size, >= 0 */
  int32_t resume;       /* continue the previous call's search state */
} dm_lbfgs_params;
dm_status dm_lbfgs_solve(dm_ctx* ctx, int32_t iters, const dm_lbfgs_params* params, int32_t msg_prec,
                         void* lambda, double* lb_trace, double* gamma_trace, int32_t* taken);

/* Subgradient of the dual (first step of Alg. 1): per multiplier, 1 where the
 * minimising assignment of its row sets the variable (exactly-one rows: the
 * smallest multiplier, lowest position on ties; +-1 rows: the fewest +1
 * entries among the minimisers, the smallest multipliers of each sign with
 * lower positions first on ties).
 *  lambda [device] (msg_prec) [nnz]; g [device] uint8 [nnz] out;
 *  *lb [host] out (the bound at lambda) or NULL.  Synchronises. */
dm_status dm_subgradient(dm_ctx* ctx, int32_t msg_prec, const void* lambda, uint8_t* g, double* lb);

/* The direction step of Alg. 1 on a given history: d^ = H g by the two-loop
 * recursion over the pairs (S[k], Y[k]), k = 0 (oldest) .. h-1 (newest), then
 * the projection to zero mean over each variable's rows.  Every pair needs
 * s^T y != 0.
 *  S [device] (msg_prec) [h * nnz]; Y [device] int8 [h * nnz] (differences of
 *  subgradients, values -1, 0, 1); g [device] uint8 [nnz]; d [device]
 *  (msg_prec) [nnz] out.  Enqueue only (allocates work buffers). */
dm_status dm_lbfgs_direction(dm_ctx* ctx, int32_t msg_prec, int32_t h, const void* S, const int8_t* Y,
                             const uint8_t* g, void* d);

/* Confident-variable fixing (Appendix "Coarse-to-fine solving strategy"):
 * at lambda, the min-marginal differences M^j_i of every free variable; a
 * variable agrees when all its M^j_i are < 0 (prefers 1) or all > 0 (prefers
 * 0); the agreeing variables are ranked by |sum_j M^j_i| (largest first, ties
 * to the lower variable) and the top floor(frac * count) are fixed to their
 * preferred values.
 *  lambda [device] (msg_prec) [nnz]; frac in [0, 1];
 *  fix [device] int8 [n_prod_tri] out: -1 free, else the value the element is
 *  fixed to (presolve fixings and the new ones); *n_agree, *n_fixed [host]
 *  out or NULL.  Synchronises. */
dm_status dm_confident_fixing(dm_ctx* ctx, int32_t msg_prec, const void* lambda, double frac, int8_t* fix,
                              int64_t* n_agree, int64_t* n_fixed);

/* Re-run presolve (integer unit propagation) from the given fixings and
 * replace the reduced problem by the residual one: later calls (multipliers,
 * dual solves, rounding, ...) work on the residual, and primal vectors still
 * cover every element, fixed ones included.  fix == NULL restores the
 * problem without fixings.  If the fixings are infeasible the problem without
 * fixings is restored and DM_ERR_INFEASIBLE returned.  Multiplier arrays of
 * the previous problem do not fit the new one (its nnz changes).
 *  fix [device] int8 [n_prod_tri] or NULL; *info [host] out (new sizes) or
 *  NULL.  Synchronises. */
dm_status dm_fix_variables(dm_ctx* ctx, const int8_t* fix, dm_space_info* info);

/* Dual objective (A8; Eq. (D)) at lambda: offset + sum over rows of the row
 * minimum (soft-min for temperature > 0).  Synchronises; *lb [host]. */
dm_status dm_lower_bound(dm_ctx* ctx, const void* lambda, double temperature, int32_t msg_prec,
                         double* lb);

/* Primal rounding (A9, A10).  On a copy of (c, lambda): sweep all rows; when
 * every free variable's min-marginal differences share one strict sign, take
 * that assignment (M < 0 -> 1, M > 0 -> 0; Appendix "Coarse-to-fine",
 * min-marginal equation) and check A x = b exactly in integers; otherwise
 * perturb the copied costs (agreeing variables pushed towards their value by
 * delta, the others by delta*u, u in [-1,1) from splitmix64(seed, round,
 * variable)), run iters_per_round Jacobi iterations and grow delta by gamma.
 * delta0 <= 0 means 0.1 * mean |M| at the first sweep.
 *  x [device] uint8 [n_prod_tri] out (fixed variables included);
 *  primal_obj, feasible, rounds_used [host] out.  A failed rounding is not an
 *  error: it returns DM_OK with *feasible = 0.  Synchronises. */
typedef struct {
  int32_t rounds;
  int32_t iters_per_round;
  double delta0;
  double gamma;
  uint64_t seed;
  double omega;
  int32_t msg_prec;
} dm_round_params;
dm_status dm_round_primal(dm_ctx* ctx, const dm_round_params* params, const void* lambda,
                          uint8_t* x, double* primal_obj, int32_t* feasible, int32_t* rounds_used);

/* Exact integer check of A x = b over every row of the full ILP; returns the
 * number of violated rows in *violations [host].  Synchronises. */
dm_status dm_check_primal(dm_ctx* ctx, const uint8_t* x, int64_t* violations);

/* Exact search on the residual of confident fixing (Appendix "Coarse-to-fine
 * solving strategy": the variables left free after fixing are solved
 * exactly; the paper uses a MILP solver there, this is the library's own
 * depth-first branch and bound).  The searched problem is the ILP with the
 * fixings base_fix (NULL: none).  Per node (base fixings plus the branching
 * decisions on its path): presolve from the node's fixings (an infeasible
 * node is pruned), dual_iters Jacobi iterations from dm_init_lambda (their
 * best bound is a valid lower bound of the node; Eq. (D)), rounding with the
 * given parameters for a primal, and the branching choice: the free
 * variable whose summed min-marginal differences are closest to zero (ties
 * to the lower variable), its preferred value (negative sum -> 1) explored
 * first.  A node is pruned when its bound is within rel_tol * max(1,
 * |incumbent|) of the incumbent.  On return the problem with base_fix is
 * in place (as after dm_fix_variables(base_fix); infeasible base fixings
 * leave the problem without fixings and status DM_SEARCH_INFEASIBLE).
 *  base_fix [device] int8 [n_prod_tri] (-1 free, else the fixed value) or
 *  NULL; x [device] uint8 [n_prod_tri] out (the best primal, zeros if none);
 *  *primal_obj [host] (+inf if none), *bound [host] (the optimum when proved,
 *  else the root bound), *nodes [host] (nodes visited), *status [host]:
 *  DM_SEARCH_OPTIMAL (tree exhausted: x is optimal within rel_tol),
 *  DM_SEARCH_INFEASIBLE (tree exhausted, no feasible x), DM_SEARCH_LIMIT
 *  (max_nodes reached: x is the best found); *info [host] out (sizes of the
 *  restored problem) or NULL.  Synchronises. */
typedef struct {
  int32_t max_nodes;       /* node limit, >= 1 */
  int32_t dual_iters;      /* Jacobi iterations per node, >= 1 */
  double omega;            /* their damping, (0, 1] */
  double rel_tol;          /* pruning tolerance, >= 0 */
  dm_round_params round;   /* rounding at each node; round.msg_prec is the
                              message precision of the whole search */
} dm_search_params;
enum { DM_SEARCH_INFEASIBLE = -1, DM_SEARCH_LIMIT = 0, DM_SEARCH_OPTIMAL = 1 };
dm_status dm_exact_search(dm_ctx* ctx, const dm_search_params* params, const int8_t* base_fix, uint8_t* x,
                          double* primal_obj, double* bound, int32_t* nodes, int32_t* status,
                          dm_space_info* info);

/* Local repair of a primal (Appendix "Coarse-to-fine solving strategy": the
 * confident part of an assignment stays fixed and the rest is solved
 * exactly, here by the exact search above).  The rows of the full ILP that x
 * violates define a neighbourhood: step 1 takes every element of those rows,
 * each further step adds the elements of the closedness rows that touch the
 * neighbourhood (projection rows, which span a face's candidates, are not
 * followed).  Every element outside the neighbourhood keeps its value in x
 * (elements fixed by presolve keep theirs), and dm_exact_search with params
 * searches the neighbourhood (to optimality, or its best primal when it
 * stops at params->max_nodes); when it finds no feasible completion the
 * neighbourhood grows by one step, up to max_hops steps.  A feasible x is
 * returned unchanged with its objective.  The problem the context held
 * before the call (with any dm_fix_variables fixings) is in place afterwards,
 * rebuilt identically, so its multiplier arrays stay valid and a
 * dm_lbfgs_solve session on it can be resumed.
 *  x [device] uint8 [n_prod_tri] in/out: the repaired assignment when one is
 *  found, else unchanged; *primal_obj [host] (+inf if none), *feasible
 *  [host], *hops_used [host] (steps of the last neighbourhood searched, 0 if
 *  x was feasible), *n_free [host] (its free elements).  Errors as
 *  dm_exact_search; DM_ERR_INVALID_ARG for max_hops < 1.  Synchronises. */
dm_status dm_repair_primal(dm_ctx* ctx, const dm_search_params* params, int32_t max_hops, uint8_t* x,
                           double* primal_obj, int32_t* feasible, int32_t* hops_used, int64_t* n_free);

/* Gradient of the smoothed bound L_T(lambda) (A11).  With
 * lambda^j_i = c_i/|J_i| + phi^j_i and phi held fixed:
 *   dL/dc_i = mean_j mu^j_i (free), 1 (fixed to 1), 0 (fixed to 0),
 * where mu^j_i is the probability of s_i = 1 under exp(-s^T lambda^j / T);
 * chained through Eq. (cost) to the descriptors with areas and candidates
 * constant.  grad_out scales the result.  gcost [device] float32
 * [n_prod_tri] out or NULL; gFX [device] float32 [nvx*D], gFY [nvy*D] out;
 * *value [host] out (L_T) or NULL.  Synchronises when value is not NULL. */
dm_status dm_smoothed_backward(dm_ctx* ctx, const void* lambda, double temperature,
                               int32_t msg_prec, double grad_out, const float* FX,
                               const float* FY, int32_t D, float* gcost, float* gFX, float* gFY,
                               double* value);

/* Mixed vertex areas (Meyer et al. 2003) of a device mesh, for checks.
 *  out [device] double [nv]. */
dm_status dm_mixed_areas(dm_ctx* ctx, const dm_mesh* M, double* out);

/* Measurement hook: while enabled, every dual-sweep kernel launch (of any
 * entry point) carries a pair of HIP events that record the kernel's own
 * start and end (hipExtLaunchKernelGGL) on the context's stream.
 * dm_timing_read synchronises the stream and returns the number of timed
 * launches and the sum of their durations in milliseconds [host], then
 * clears the record.  Off by default. */
dm_status dm_timing_enable(dm_ctx* ctx, int32_t enable);
dm_status dm_timing_read(dm_ctx* ctx, int64_t* launches, double* total_ms);

/* Version string of the library build. */
const char* dm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DISCOMATCH_H */
