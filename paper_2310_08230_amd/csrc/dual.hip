// Jacobi min-marginal averaging on the Lagrangean dual (Sec. 3.2, Eq. (D);
// the MMA step of Alg. 1) and the dual bound.
//
// State layout.  The multipliers lambda^j_i of free variable i live in one
// record of REC reals: slots 0-2 for its three closedness rows (edges k = 0,
// 1, 2 of the element), slot 3 for its first projection row, slot 4 for its
// Y projection row when the element is triangle-triangle, slot 5 for the cost
// c_i, slot 6 for its number of rows (a generic problem's variable takes slots
// 0 to |J_i| - 1 in row order).  Two record buffers alternate between
// iterations.
//
// One iteration is one kernel launch over every row of the presolved problem:
//   1. each entry reads its variable's record from the previous iteration and
//      restores dual feasibility, lambda^j_i = s_j + (c_i - sum_k s_k)/|J_i|;
//   2. each row computes its minimum and the min-marginal differences
//      M^j_i = min_{s_i=1} - min_{s_i=0} (Appendix "Coarse-to-fine");
//   3. each entry writes s_j' = lambda^j_i - omega M^j_i to the other buffer;
//   4. row minima are summed into an FP64 bound in a fixed order.
// Steps 1 and 3 together are lambda <- lambda - omega (M - mean_j M): the
// mean of the min-marginals is exactly what the projection in step 1 adds
// back, so the variable-averaging pass needs no separate launch.
//
// Rows: closedness rows (short, coefficients +-1, right-hand side b) are packed
// into chunks of at most 255 entries, one 256-thread block per chunk, with the
// row minimum from sorted prefix sums in LDS: choosing k entries with
// coefficient +1 and k-b with -1 costs at least S+(k) + S-(k-b), the sums of
// the k and k-b smallest multipliers.  Projection rows (all +1, b = 1) get one
// block each and reduce (min, argmin, second min) across the block.  With a
// temperature T > 0 every min becomes the soft-min -T log sum exp(-./T); short
// rows then run a partial-sum recursion with one lane per partial sum.
#include <hip/hip_ext.h>

#include <cmath>

#include "dm_internal.h"

namespace {

constexpr int MODE_UPDATE = SWEEP_UPDATE, MODE_EVAL = SWEEP_EVAL, MODE_BOUND = SWEEP_BOUND,
              MODE_SUBGRAD = SWEEP_SUBGRAD;

template <typename R>
__device__ inline R rinf() {
  return R(INFINITY);
}

template <typename R>
__device__ inline R r_exp(R x);
template <>
__device__ inline float r_exp<float>(float x) { return expf(x); }
template <>
__device__ inline double r_exp<double>(double x) { return exp(x); }
template <typename R>
__device__ inline R r_log(R x);
template <>
__device__ inline float r_log<float>(float x) { return logf(x); }
template <>
__device__ inline double r_log<double>(double x) { return log(x); }
template <typename R>
__device__ inline R r_log1p(R x);
template <>
__device__ inline float r_log1p<float>(float x) { return log1pf(x); }
template <>
__device__ inline double r_log1p<double>(double x) { return log1p(x); }

// soft-min of two values (hard min when T == 0):
// -T log(e^{-a/T} + e^{-b/T}) = min(a, b) - T log1p(e^{-|a-b|/T})
template <typename R, bool SOFT>
__device__ inline R smin2(R a, R b, R T) {
  if (!SOFT) return a < b ? a : b;
  if (a == rinf<R>()) return b;
  if (b == rinf<R>()) return a;
  const R m = a < b ? a : b, d = a < b ? b - a : a - b;
  return m - T * r_log1p<R>(r_exp<R>(-d / T));
}

// Scaled soft-min arithmetic for the short-row recursion.  Values are kept in
// units u = x / (T ln 2) (FP32) or u = x / T (FP64), so that the soft-min of
// two values is min - L(1 + E(-|a - b|)) and of many min - L(sum E(u - min))
// with E = 2^x, L = log2 (FP32: the hardware exp2 / log2 instructions, about
// one ulp) or E = exp, L = log (FP64).
template <typename R>
struct SoftUnits;
template <>
struct SoftUnits<float> {
  static constexpr float big = 3.40282347e+38f;   // largest finite value
  static __device__ float unit(float T) { return T * 0.693147180559945309f; }   // x = u * unit
  static __device__ float E(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ float L(float x) { return __builtin_amdgcn_logf(x); }
  static __device__ float L1p(float x) { return __builtin_amdgcn_logf(1.0f + x); }
};
template <>
struct SoftUnits<double> {
  static constexpr double big = 1.7976931348623157e+308;
  static __device__ double unit(double T) { return T; }
  static __device__ double E(double x) { return exp(x); }
  static __device__ double L(double x) { return log(x); }
  static __device__ double L1p(double x) { return log1p(x); }
};

// soft-min of two values in scaled units, without branches: with the smaller
// value clamped to the largest finite one, an infinite larger value gives
// E(-inf) = 0 and the result is the smaller value (inf when both are inf)
template <typename R>
__device__ inline R smin2u(R a, R b) {
  // with both operands clamped to the largest finite value, -|a - b| is the
  // exponent m - M of two finite values, -huge when one is infinite and 0
  // when both are (then m is inf and so is the result)
  const R ac = fmin(a, SoftUnits<R>::big), bc = fmin(b, SoftUnits<R>::big);
  return fmin(a, b) - SoftUnits<R>::L1p(SoftUnits<R>::E(-fabs(ac - bc)));
}

// One DPP lane move (a VALU operation): ctrl 0xB1 swaps neighbours (quad
// permutation 1,0,3,2), 0x4E swaps pairs (2,3,0,1), 0x141 mirrors each group of
// eight lanes, 0x140 each row of sixteen; 0x138 shifts the whole wave by one
// lane (lane i reads lane i - 1), 0x130 the other way (lane i reads i + 1).
// A lane whose source is missing reads 0; callers mask those lanes.
template <int CTRL, typename R>
__device__ inline R dpp_move(R v) {
  if constexpr (sizeof(R) == 4) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
  } else {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(bits & 0xFFFFFFFFll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(int(bits >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | (static_cast<long long>(lo) & 0xFFFFFFFFll));
  }
}

// min / sum over the W lanes (W = 8, 16 or 32) of an aligned segment, the same
// value in every lane: DPP steps within each sixteen-lane row (every pairing
// is symmetric, so all lanes form the same sums), one shuffle joins two rows
// min of v and its DPP-moved copy (values are never NaN); adding +0 to the
// moved value (-0 becomes +0, nothing else changes) gives an arithmetic
// result, which needs no NaN canonicalisation before the min, and the move
// folds into that add
template <int CTRL, typename R>
__device__ inline R min_dpp(R v) {
  return fmin(v, dpp_move<CTRL, R>(v) + R(0));
}

// FP32 values as integers of the same order (the sign-magnitude bits with
// the magnitude flipped for negative values; every non-NaN value, infinities
// included, keeps its place), so a segment minimum runs on integer DPP mins,
// which need no NaN canonicalisation of the moved operand
__device__ inline int32_t ordered_bits(float f) {
  const int32_t i = __float_as_int(f);
  return i ^ ((i >> 31) & 0x7FFFFFFF);
}
__device__ inline float from_ordered_bits(int32_t k) { return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF)); }

template <int CTRL>
__device__ inline int32_t imin_dpp(int32_t v) {
  const int32_t o = __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
  return o < v ? o : v;
}

// ordered bits of the FP32 segment minimum
template <int W>
__device__ inline int32_t seg_min_bits(float v) {
  int32_t k = ordered_bits(v);
  k = imin_dpp<0xB1>(k);
  k = imin_dpp<0x4E>(k);
  k = imin_dpp<0x141>(k);
  if constexpr (W >= 16) k = imin_dpp<0x140>(k);
  if constexpr (W == 32) {
    const int32_t o = __shfl_xor(k, 16, 32);
    k = o < k ? o : k;
  }
  return k;
}

template <int W, typename R>
__device__ inline R seg_min(R v) {
  if constexpr (sizeof(R) == 4) {
    return from_ordered_bits(seg_min_bits<W>(v));
  } else {
    v = min_dpp<0xB1>(v);
    v = min_dpp<0x4E>(v);
    v = min_dpp<0x141>(v);
    if constexpr (W >= 16) v = min_dpp<0x140>(v);
    if constexpr (W == 32) v = fmin(v, __shfl_xor(v, 16, 32) + R(0));
    return v;
  }
}

template <int W, typename R>
__device__ inline R seg_sum(R v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  if constexpr (W >= 16) v += dpp_move<0x140>(v);
  if constexpr (W == 32) v += __shfl_xor(v, 16, 32);
  return v;
}

// soft-min over the W lanes of a segment in scaled units, as the two parts
// every lane gets: the hard minimum mc and the sum e of one exponential per
// lane; the soft-min is mc - L(e), left to the caller so that only the lane
// that needs it takes the logarithm.  With the minimum clamped to the largest
// finite value, lanes holding inf add E(-inf) = 0, and a segment of infs
// gives L(0) = -inf, so inf.
template <int W, typename R>
__device__ inline void seg_softmin_parts(R x, R& mc, R& e) {
  if constexpr (sizeof(R) == 4) {   // the clamp on the ordered bits: no NaN canonicalisation
    mc = from_ordered_bits(min(seg_min_bits<W>(x), ordered_bits(SoftUnits<R>::big)));
  } else {
    const R m = seg_min<W, R>(x);
    mc = m < SoftUnits<R>::big ? m : SoftUnits<R>::big;
  }
  e = seg_sum<W, R>(SoftUnits<R>::E(mc - x));
}

// multiplier of entry word w from the previous record buffer, with dual
// feasibility restored
template <typename R>
__device__ inline R cur_lambda(const R* __restrict__ rec, uint32_t w) {
  R lam[5];
  rec_lambdas<R>(rec, size_t(w & W_VAR_MASK), lam);
  const int k = int((w >> W_SLOT_SHIFT) & 7u);
  return k == 0 ? lam[0] : k == 1 ? lam[1] : k == 2 ? lam[2] : k == 3 ? lam[3] : lam[4];
}

template <typename R>
__device__ inline void write_out(R* __restrict__ out, uint32_t w, R v) {
  out[size_t(w & W_VAR_MASK) * REC + ((w >> W_SLOT_SHIFT) & 7u)] = v;
}

// block-wide FP64 sum of a 256-thread block in a fixed order: an xor butterfly
// inside each wave (every lane ends with the same value, since a + b == b + a
// exactly), then the four wave sums in index order
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return r;
}

// Each block stores the sum of its row minima; the per-block partials of one
// launch are summed in index order by block 0 of the next launch (the kernel
// boundary makes them visible without atomics or cache maintenance) or by a
// one-block kernel after the last launch.
__device__ inline void store_partial(double part, double* partial, int32_t item) {
  if (threadIdx.x == 0) partial[item] = part;
}

__device__ inline void reduce_partials(const double* partial, int n, double offset, double* out, double* red) {
  const double tot = sum_partials_256(partial, n, red);
  if (threadIdx.x == 0) *out = offset + tot;
}

struct SweepArgs {
  const uint32_t* word;
  const int32_t* rrow_ptr;
  const int32_t* soft_row;  // short rows in order of length (smoothed form)
  int32_t soft_c8, soft_c16;  // short rows of at most 7 / of 8 to 15 entries
  const int32_t* rrow_b;
  const int4* chunk_desc;   // (first row, rows, first entry, entries) per chunk
  const unsigned long long* chunk_mask;   // bit e: entry e of the chunk starts a row
  const uint32_t* chunk_word;   // 64 words per chunk, CHUNK_PAD past its end
  const int8_t* chunk_b;        // 64 per chunk: right-hand side of the entry's row
  int32_t n_short_blocks;   // items of short rows (hard form: row tiles, then chunks)
  int32_t n_tile_items;     // hard form: blocks of four 64-row tiles
  int32_t n_tiles;
  const uint32_t* tile_word;  // per tile: 16 x 64 entry words (slot j of lane l at j * 64 + l), CHUNK_PAD
  int32_t n_short;
  int32_t n_rows;
  int32_t n_items;          // short-row blocks + long-row blocks
  int32_t n_chunks;         // wave chunks of short rows (hard form)
  int32_t long_wpr;         // waves per projection row: 1 or 4
  int32_t n_long;           // projection rows
  const int32_t* long_perm; // projection rows (relative to n_short) in launch order
  const int32_t* xcd_item;  // hard form: item of block b at (b % 8) * xcd_stride + b / 8, or -1
  int32_t xcd_stride;
  double* partial;          // this launch's per-block partials
  const double* prev_partial; // previous launch's partials still to be summed, or NULL
  int32_t prev_n;
  double prev_offset;
  double* prev_out;
  // quasi-Newton extensions (hard min only): rows see lambda + gamma * dir
  // when dir is set (dir in slot planes: slot k of variable i at
  // k * plane + i; gamma a device scalar); the launch does nothing when
  // *skip is nonzero; MODE_SUBGRAD writes the row's minimising assignment
  // (1 / 0 per entry) to gsub in the same slot planes
  int64_t plane;
  const void* dir;
  const double* gamma;
  const int32_t* skip;
  uint8_t* gsub;
};

__device__ inline size_t slot_index(const SweepArgs& A, uint32_t w) {
  return size_t((w >> W_SLOT_SHIFT) & 7u) * size_t(A.plane) + size_t(w & W_VAR_MASK);
}

// multiplier seen by the rows: the record's, moved along dir when one is set
template <typename R>
__device__ inline R row_lambda(const SweepArgs& A, const R* __restrict__ rin, uint32_t w, R gam) {
  R v = cur_lambda<R>(rin, w);
  if (A.dir) v += gam * static_cast<const R*>(A.dir)[slot_index(A, w)];
  return v;
}

// ---------------------------------------------------------------- short rows, hard min
// One wave per chunk of whole closedness rows (<= 64 entries, one per lane),
// four chunks per block, no LDS and no barrier until the bound.  Every
// cross-lane step runs in a wave-uniform loop, so no lane ever reads from an
// inactive lane:
//  1. lane e holds entry e (multiplier, sign, word); the first lanes hold the
//     row starts, and each lane finds its row with a 5-step binary search;
//  2. rank inside the row's sign group by comparing with the row's lanes;
//  3. ds_permute moves every value to its sorted position;
//  4. a segmented inclusive scan gives S(k), the sum of the k smallest of a
//     group, at the lane of the k-th smallest;
//  5. each lane evaluates its two constrained minima over k.
// 16-byte LDS read of four FP32 or two FP64 values
template <typename R>
struct LdsVec;
template <>
struct LdsVec<float> {
  using type = float4;
  static __device__ float get(const float4& v, int u) { return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w; }
};
template <>
struct LdsVec<double> {
  using type = double2;
  static __device__ double get(const double2& v, int u) { return u == 0 ? v.x : v.y; }
};

template <typename R>
__device__ inline R permute_to(int dst_lane, R v) {   // push v to lane dst_lane
  if constexpr (sizeof(R) == 4) {
    return __int_as_float(__builtin_amdgcn_ds_permute(dst_lane << 2, __float_as_int(v)));
  } else {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_permute(dst_lane << 2, int(bits & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_ds_permute(dst_lane << 2, int(bits >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | (static_cast<long long>(lo) & 0xFFFFFFFFll));
  }
}

template <typename R, int MODE>
__device__ inline double short_chunk_hard(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out,
                                          R omega, R gam, int32_t wc, R* wave_vals) {
  const int lane = threadIdx.x & 63;
  double rowpart = 0.0;
  if (wc < A.n_chunks) {   // uniform across the wave
    // the padded chunk: words and right-hand sides straight from the chunk index
    const unsigned long long starts = A.chunk_mask[wc];
    const uint32_t wp = A.chunk_word[size_t(wc) * 64 + lane];
    const int32_t b = A.chunk_b[size_t(wc) * 64 + lane];
    const bool act = wp != CHUNK_PAD;
    const uint32_t w = act ? wp : 0u;
    const int32_t ne = __popcll(__ballot(act));
    const R lam = act ? row_lambda<R>(A, rin, w, gam) : R(0);
    const int g = int(w >> 31);
    // my row from the chunk's row-start mask: its start is the last set bit at
    // or below this lane, its end the next set bit (or the chunk's end)
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const unsigned long long below = starts & le, above = starts & ~le;
    const int32_t s = 63 - __clzll(static_cast<long long>(below));   // entry 0 always starts a row
    const int32_t n = (above ? __ffsll(static_cast<long long>(above)) - 1 : ne) - s;

    const unsigned long long negm = __ballot(act && g);
    const unsigned long long rowm = act ? (((n >= 64) ? ~0ull : ((1ull << n) - 1ull)) << s) : 0ull;
    const int32_t P = __popcll(rowm & ~negm);
    const int32_t N = n - P;
    // rank of this entry in its sign group (ties broken by lane): the wave's
    // values go to its own 64-entry LDS slice, and each lane reads its row in
    // aligned 16-byte pieces (lanes of one row read the same addresses: a
    // broadcast); only this wave touches the slice, so a wave-level fence
    // orders the writes before the reads
    wave_vals[lane] = lam;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int V = 16 / int(sizeof(R));   // values per 16-byte read
    using Vec = typename LdsVec<R>::type;
    if (__ballot(act && b != 0) == 0ull) {   // uniform: every row of the chunk has b = 0
      // Rows with b = 0 choose k entries of each sign.  With P and Q the
      // sorted +1 and -1 groups, the pair sums p_(j) + q_(j) never decrease,
      // so the minimiser takes the k* pairs with negative sums.  An entry of
      // rank r (1-based, ties by lane) is taken iff the other group holds at
      // least r values whose sum with it is negative.  Its min-marginal needs
      // only the order statistics around k*: with U = min(p_(k*+1), -q_(k*))
      // and V = min(q_(k*+1), -p_(k*)) (empty terms +inf),
      //   taken +1: p - U,  left +1: p + V,  taken -1: q - V,  left -1: q + U,
      // and the row minimum is the sum of the taken values.
      int32_t rank = 0, cnt = 0;
      if (act) {
        const R nlam = -lam;
        for (int a = s & ~(V - 1); a < s + n; a += V) {
          const Vec v = *reinterpret_cast<const Vec*>(wave_vals + a);
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int src = a + u;
            const R lq = LdsVec<R>::get(v, u);
            const int gq = int((negm >> src) & 1ull);
            if (src >= s && src < s + n) {
              if (gq == g) rank += (lq < lam) || (lq == lam && src < lane);
              else cnt += lq < nlam;
            }
          }
        }
      }
      const bool sel = act && cnt > rank;
      // U collects left +1 and taken -1 entries, V left -1 and taken +1
      // entries, each as +-lambda
      const R t = sel ? -lam : lam;
      R* uvals = wave_vals + 64;
      R* vvals = wave_vals + 128;
      uvals[lane] = (act && g == int(sel)) ? t : rinf<R>();
      vvals[lane] = (act && g != int(sel)) ? t : rinf<R>();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (act) {
        R U = rinf<R>(), Vv = rinf<R>();
        if (MODE == MODE_UPDATE || MODE == MODE_EVAL) {
          for (int a = s & ~(V - 1); a < s + n; a += V) {
            const Vec uv = *reinterpret_cast<const Vec*>(uvals + a);
            const Vec vv = *reinterpret_cast<const Vec*>(vvals + a);
#pragma unroll
            for (int u = 0; u < V; ++u) {
              const int src = a + u;
              if (src >= s && src < s + n) {
                U = fmin(U, LdsVec<R>::get(uv, u));
                Vv = fmin(Vv, LdsVec<R>::get(vv, u));
              }
            }
          }
          const R Wm = g == int(sel) ? Vv : U;
          const R M = sel ? lam - Wm : lam + Wm;
          if (MODE == MODE_UPDATE) write_out<R>(out, w, lam - omega * M);
          if (MODE == MODE_EVAL) write_out<R>(out, w, M);
        }
        if (MODE == MODE_SUBGRAD) A.gsub[slot_index(A, w)] = uint8_t(sel ? 1 : 0);
        if (sel) rowpart = double(lam);
      }
      return rowpart;
    }
    // general right-hand sides: the rank as above, then a sort of the chunk
    int32_t rank = 0;
    if (act) {
      for (int a = s & ~(V - 1); a < s + n; a += V) {   // a + V <= 64: the slice's end
        const Vec v = *reinterpret_cast<const Vec*>(wave_vals + a);
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int src = a + u;
          const R lq = LdsVec<R>::get(v, u);
          const int gq = int((negm >> src) & 1ull);
          if (src >= s && src < s + n && gq == g) rank += (lq < lam) || (lq == lam && src < lane);
        }
      }
    }
    // sorted position: positive group first, then negative group
    const int dst = act ? s + (g ? P + rank : rank) : lane;
    const R srt = permute_to<R>(dst, lam);
    // segmented inclusive scan over the sorted groups: lane j of row [s, s+n)
    // belongs to the +1 group if j - s < P
    const int32_t seg = act ? s + (lane - s < P ? 0 : P) : lane;
    R pre = srt;
    for (int off = 1; off < 64; off <<= 1) {
      const R t = __shfl(pre, lane >= off ? lane - off : 0);
      if (lane - off >= seg) pre += t;
    }
    // pre at lane (group start + k - 1) = S_group(k).
    // Choosing k of the own group and k - bb of the other costs
    // f(k) = S_own(k) + S_oth(k - bb) for k in [klo, khi]; its increments
    // o_k + q_{k-bb} (sorted values of the two groups) never decrease, so f is
    // convex and its smallest minimiser is klo plus the number of negative
    // increments.  The constrained minima of an entry at sorted position t are
    // minima of two more convex sequences over ranges that depend on t:
    //   A(k) = S_own(k-1) + S_oth(k-bb)  (increments o_{k-1} + q_{k-bb}),
    //   B(k) = S_own(k+1) + S_oth(k-bb)  (increments o_{k+1} + q_{k-bb}),
    // so they too come from counts of negative increments, clamped to the range.
    // 1. sorted role: lane L holds the k-th smallest of its group
    const int32_t j = lane - s;
    const int gs = act && j >= P;
    const int32_t ks = j - (gs ? P : 0) + 1;
    const int32_t own_s = gs ? N : P, oth_s = gs ? P : N, bb_s = gs ? -b : b;
    const int32_t klo_s = bb_s > 0 ? bb_s : 0;
    const int32_t khi_s = own_s < oth_s + bb_s ? own_s : oth_s + bb_s;
    const int32_t qi = s + (gs ? 0 : P) + (ks - bb_s) - 1;
    const R qv = __shfl(srt, qi >= 0 && qi < 64 ? qi : 0);
    const R om1 = __shfl(srt, lane > 0 ? lane - 1 : 0);
    const R op1 = __shfl(srt, lane < 63 ? lane + 1 : 63);
    const int32_t alo_s = klo_s > 1 ? klo_s : 1;
    const int32_t bhi_s = khi_s < own_s - 1 ? khi_s : own_s - 1;
    const unsigned long long mF = __ballot(act && ks > klo_s && ks <= khi_s && srt + qv < R(0));
    const unsigned long long mA = __ballot(act && ks > alo_s && ks <= khi_s && om1 + qv < R(0));
    const unsigned long long mB = __ballot(act && ks > klo_s && ks <= bhi_s && op1 + qv < R(0));
    // 2. entry role: this lane's entry has own-group position t = rank + 1
    const int32_t own = g ? N : P, oth = g ? P : N, bb = g ? -b : b;
    const int32_t obase = s + (g ? P : 0), tbase = s + (g ? 0 : P);
    const int32_t klo = bb > 0 ? bb : 0;
    const int32_t khi = own < oth + bb ? own : oth + bb;
    const unsigned long long gmask = act ? (((own >= 64) ? ~0ull : ((1ull << own) - 1ull)) << obase) : 0ull;
    const int32_t kbest = klo + __popcll(mF & gmask);   // smallest minimiser
    auto s_own = [&](int32_t k) {   // every lane shuffles; k == 0 gives 0
      const int i = obase + k - 1;
      const R v = __shfl(pre, i >= 0 && i < 64 ? i : 0);
      return k <= 0 ? R(0) : v;
    };
    auto s_oth = [&](int32_t k) {
      const int i = tbase + k - 1;
      const R v = __shfl(pre, i >= 0 && i < 64 ? i : 0);
      return k <= 0 ? R(0) : v;
    };
    const R rmin = s_own(kbest) + s_oth(kbest - bb);
    R m1 = rmin, m0 = rmin;
    if (MODE == MODE_UPDATE || MODE == MODE_EVAL) {
      const int32_t t = rank + 1;
      const bool sel = t <= kbest;   // the minimiser takes this entry
      // the other side's minimum: f at the nearest k on that side, and A or B
      // at their convex minimiser clamped to the side's range
      const int32_t x1 = sel ? t - 1 : t;
      const bool c1ok = sel ? (t - 1 >= klo) : (t <= khi);
      const R c1 = s_own(x1) + s_oth(x1 - bb);
      int32_t lo2, hi2, kst;
      if (sel) {
        lo2 = t > klo ? t : klo;
        hi2 = khi < own - 1 ? khi : own - 1;
        kst = klo + __popcll(mB & gmask);
      } else {
        lo2 = klo > 1 ? klo : 1;
        hi2 = t - 1 < khi ? t - 1 : khi;
        kst = lo2 + __popcll(mA & gmask);
      }
      const bool c2ok = lo2 <= hi2;
      const int32_t k2 = kst < lo2 ? lo2 : (kst > hi2 ? hi2 : kst);
      const R so2 = s_own(sel ? k2 + 1 : k2 - 1);
      const R st2 = s_oth(k2 - bb);
      const R c2 = sel ? (so2 - lam) + st2 : (lam + so2) + st2;
      R other = rinf<R>();
      if (c1ok) other = c1;
      if (c2ok && c2 < other) other = c2;
      if (sel) m0 = other;
      else m1 = other;
    }
    if (act) {
      const R M = m1 - m0;
      if (MODE == MODE_UPDATE) write_out<R>(out, w, lam - omega * M);
      if (MODE == MODE_EVAL) write_out<R>(out, w, M);
      if (MODE == MODE_SUBGRAD)
        A.gsub[slot_index(A, w)] = uint8_t(rank < kbest ? 1 : 0);
      if (lane == s) rowpart = double(rmin);
    }
  }
  return rowpart;
}

// the four waves of a block take four adjacent chunks
template <typename R, int MODE>
__device__ void short_wave_hard(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out, R omega,
                                R gam, unsigned char* smem, double* red, int32_t item) {
  const int wave = threadIdx.x >> 6;
  R* wave_vals = reinterpret_cast<R*>(smem) + wave * 192;   // three 64-value slices per wave
  const int32_t wc = (item - A.n_tile_items) * 4 + wave;
  const double rowpart = short_chunk_hard<R, MODE>(A, rin, out, omega, gam, wc, wave_vals);
  double part = block_sum(rowpart, red);
  store_partial(part, A.partial, item);
}

// ---------------------------------------------------------------- short rows with b = 0, one lane per row
// Rows with right-hand side 0 and at most TILE_HALF entries of each sign run
// one lane per row, 64 rows per wave (a tile): the row's +1 entries sit in
// slots 0 to TILE_HALF - 1 and its -1 entries in the next TILE_HALF slots,
// each group in row order; slot j of lane l is word j * 64 + l of the tile,
// CHUNK_PAD where the group has ended.  The multipliers stay in registers and
// the closed form of the b = 0 rows (see short_chunk_hard) is evaluated over
// pairs: within a group the earlier entry's rank rises if it is larger, the
// later one's if it is not smaller; across the groups both counts rise if the
// pair sums to a negative value.  d = count - rank decides whether an entry
// is taken (d > 0).  A missing entry holds +inf: it is never taken, never
// ranked before a value and never pairs to a negative sum.
constexpr int TILE_HALF = 8;

// a multiplier record as loaded (two 16-byte loads for FP32, four for FP64)
template <typename R>
struct RecRaw;
template <>
struct RecRaw<float> {
  float4 lo, hi;
  __device__ void load(const float* __restrict__ rec, uint32_t i) {
    lo = *reinterpret_cast<const float4*>(rec + size_t(i) * REC);
    hi = *reinterpret_cast<const float4*>(rec + size_t(i) * REC + 4);
  }
  // lambda of slot k with dual feasibility restored, in the arithmetic of rec_lambdas
  __device__ float lambda(int k) const {
    const float sum = (((lo.x + lo.y) + lo.z) + lo.w) + hi.x;
    const float corr = (hi.y - sum) * hi.z;
    const float sk = k == 0 ? lo.x : k == 1 ? lo.y : k == 2 ? lo.z : k == 3 ? lo.w : hi.x;
    return sk + corr;
  }
};
template <>
struct RecRaw<double> {
  double2 a, b, c, d;
  __device__ void load(const double* __restrict__ rec, uint32_t i) {
    const double* r = rec + size_t(i) * REC;
    a = *reinterpret_cast<const double2*>(r);
    b = *reinterpret_cast<const double2*>(r + 2);
    c = *reinterpret_cast<const double2*>(r + 4);
    d = *reinterpret_cast<const double2*>(r + 6);
  }
  __device__ double lambda(int k) const {
    const double sum = (((a.x + a.y) + b.x) + b.y) + c.x;
    const double corr = (c.y - sum) * d.x;
    const double sk = k == 0 ? a.x : k == 1 ? a.y : k == 2 ? b.x : k == 3 ? b.y : c.x;
    return sk + corr;
  }
};

// TB: FP32 records in flight per batch (8 or 16); every load of a batch is
// issued before the first one is used (a missing entry loads record 0 and is
// then replaced).  FP64 records are twice as wide and go two at a time.
template <typename R, int MODE, int TB>
__device__ inline double tile_rows(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out, R omega,
                                   R gam, const uint32_t* __restrict__ tw) {
  constexpr int H = TILE_HALF;
  constexpr int B = sizeof(R) == 4 ? TB : 2;
  const int lane = threadIdx.x & 63;
  uint32_t wv[2 * H];
#pragma unroll
  for (int j = 0; j < 2 * H; ++j) wv[j] = tw[j * 64 + lane];
  R lam[2 * H];   // slots 0 to H - 1: +1 entries, H to 2H - 1: -1 entries
#pragma unroll
  for (int j0 = 0; j0 < 2 * H; j0 += B) {
    RecRaw<R> raw[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const uint32_t w = wv[j0 + u] != CHUNK_PAD ? wv[j0 + u] : 0u;
      raw[u].load(rin, w & W_VAR_MASK);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const uint32_t w = wv[j0 + u];
      lam[j0 + u] = w != CHUNK_PAD ? raw[u].lambda(int((w >> W_SLOT_SHIFT) & 7u)) : rinf<R>();
    }
  }
  if (A.dir) {   // uniform: rows see lambda + gamma * dir
    R dv[2 * H];
#pragma unroll
    for (int j = 0; j < 2 * H; ++j)
      dv[j] = static_cast<const R*>(A.dir)[slot_index(A, wv[j] != CHUNK_PAD ? wv[j] : 0u)];
#pragma unroll
    for (int j = 0; j < 2 * H; ++j)
      if (wv[j] != CHUNK_PAD) lam[j] += gam * dv[j];
  }
  R* lp = lam;
  R* lq = lam + H;
  int32_t d[2 * H];
#pragma unroll
  for (int j = 0; j < 2 * H; ++j) d[j] = 0;
  int32_t* dp = d;
  int32_t* dq = d + H;
#pragma unroll
  for (int j = 1; j < H; ++j)
#pragma unroll
    for (int k = 0; k < j; ++k) {
      const bool lep = lp[k] <= lp[j], leq = lq[k] <= lq[j];   // k is earlier: a tie ranks j after k
      dp[j] -= lep ? 1 : 0;
      dp[k] -= lep ? 0 : 1;
      dq[j] -= leq ? 1 : 0;
      dq[k] -= leq ? 0 : 1;
    }
#pragma unroll
  for (int j = 0; j < H; ++j)
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int ng = lp[j] + lq[k] < R(0) ? 1 : 0;   // the pair's sum (its sign is exact)
      dp[j] += ng;
      dq[k] += ng;
    }
  // U: left +1 and taken -1 entries, V: left -1 and taken +1 entries (as +-lambda)
  R U = rinf<R>(), V = rinf<R>();
  double rowmin = 0.0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    if (dp[j] > 0) {
      V = fmin(V, -lp[j]);
      rowmin += double(lp[j]);
    } else {
      U = fmin(U, lp[j]);
    }
    if (dq[j] > 0) {
      U = fmin(U, -lq[j]);
      rowmin += double(lq[j]);
    } else {
      V = fmin(V, lq[j]);
    }
  }
  if (MODE == MODE_UPDATE || MODE == MODE_EVAL || MODE == MODE_SUBGRAD) {
#pragma unroll
    for (int j = 0; j < 2 * H; ++j) {
      const uint32_t w = wv[j];
      if (w == CHUNK_PAD) continue;
      const bool neg = j >= H;
      const R lv = lam[j];
      const bool sel = d[j] > 0;
      if (MODE == MODE_SUBGRAD) {
        A.gsub[slot_index(A, w)] = uint8_t(sel ? 1 : 0);
      } else {
        // taken +1: p - U, left +1: p + V, taken -1: q - V, left -1: q + U
        const R Wm = neg == sel ? V : U;
        const R M = sel ? lv - Wm : lv + Wm;
        if (MODE == MODE_UPDATE) write_out<R>(out, w, lv - omega * M);
        if (MODE == MODE_EVAL) write_out<R>(out, w, M);
      }
    }
  }
  return rowmin;
}

template <typename R, int MODE, int TB>
__device__ void tile_block(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out, R omega, R gam,
                           double* red, int32_t item) {
  const int32_t t = item * 4 + int32_t(threadIdx.x >> 6);
  double rowpart = 0.0;
  if (t < A.n_tiles)   // uniform across the wave
    rowpart = tile_rows<R, MODE, TB>(A, rin, out, omega, gam, A.tile_word + size_t(t) * (2 * TILE_HALF * 64));
  const double part = block_sum(rowpart, red);
  store_partial(part, A.partial, item);
}

// ---------------------------------------------------------------- short rows, soft min
// One W-lane segment per row (W = 8, 16, 32 for rows of at most 7, 15, 24
// entries; the rows are taken in order of length from soft_row; a block holds
// soft_rpb<W>() rows, so the forward table fits SOFT_FTAB values); lane j holds
// the partial sum sigma = j - N of the recursion
// F_{l+1}(sigma) = smin(F_l(sigma), F_l(sigma - a_l) + lam_l),
// B_l(sigma) = smin(B_{l+1}(sigma), B_{l+1}(sigma + a_l) + lam_l).
// Rows [row0, row1) of soft_row belong to this width; blk counts the blocks of
// this width, item is the block's index among all blocks.
template <int W>
constexpr int soft_rpb() {   // rows per 256-thread block
  return W == 32 ? 4 : 256 / W;
}
template <int W>
constexpr int soft_nmax() {  // entries per row at most
  return W == 32 ? SOFT_MAX_ROW : W - 1;
}
// forward-table values per block: the largest of the three widths
constexpr int SOFT_FTAB = 16 * 15 * 16;
static_assert(soft_rpb<8>() * soft_nmax<8>() * 8 <= SOFT_FTAB && soft_rpb<32>() * soft_nmax<32>() * 32 <= SOFT_FTAB,
              "forward table too small");

template <typename R, int MODE, int W>
__device__ void short_rows_soft(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out, R omega,
                                R T, unsigned char* smem, double* red, int32_t item, int32_t blk, int32_t row0,
                                int32_t row1) {
  constexpr int RPB = soft_rpb<W>(), NMAX = soft_nmax<W>();
  const int seg = threadIdx.x / W, lane = threadIdx.x % W;
  R* Ftab = reinterpret_cast<R*>(smem) + seg * (NMAX * W);
  R* lamL = reinterpret_cast<R*>(smem) + SOFT_FTAB + seg * W;
  int8_t* aL = reinterpret_cast<int8_t*>(reinterpret_cast<R*>(smem) + SOFT_FTAB + 256) + seg * W;
  const int32_t r = row0 + blk * RPB + seg;
  const bool act = seg < RPB && r < row1;
  int32_t s = 0, n = 0, b = 0;
  uint32_t w = 0;
  R mylam = R(0);
  const R unit = SoftUnits<R>::unit(T), inv_unit = R(1) / unit;
  if (act) {
    const int32_t j = A.soft_row[r];
    s = A.rrow_ptr[j];
    n = A.rrow_ptr[j + 1] - s;
    b = A.rrow_b[j];
    if (lane < n) {
      w = A.word[s + lane];
      mylam = cur_lambda<R>(rin, w);
      lamL[lane] = mylam * inv_unit;
      aL[lane] = (w >> 31) ? int8_t(-1) : int8_t(1);
    }
  }
  __syncthreads();
  double rowpart = 0.0;
  if (act) {
    int32_t N = 0;
    for (int32_t l = 0; l < n; ++l) N += aL[l] < 0;
    const int32_t P = n - N;
    const int32_t sigma = lane - N;
    const bool valid = lane <= P + N;
    R F = (valid && sigma == 0) ? R(0) : rinf<R>();
    for (int32_t l = 0; l < n; ++l) {
      Ftab[l * W + lane] = F;   // read back below by the same lane only
      const int a = aL[l];
      const R from_lo = dpp_move<0x138>(F), from_hi = dpp_move<0x130>(F);   // F[lane - 1], F[lane + 1]
      R sh = a > 0 ? from_lo : from_hi;                                       // F[lane - a]
      if ((unsigned(lane - a) >= unsigned(W)) | !valid) sh = rinf<R>();
      F = smin2u<R>(F, sh + lamL[l]);
      if (!valid) F = rinf<R>();
    }
    R Bv = (valid && sigma == b) ? R(0) : rinf<R>();
    // lane l keeps the parts of its entry's two soft-mins (x_l = 1 and
    // x_l = 0); the logarithms are taken once, after the recursion
    R m1 = R(0), e1 = R(1), m0 = R(0), e0 = R(1);
    for (int32_t l = n - 1; l >= 0; --l) {
      const int a = aL[l];
      const R Fl = Ftab[l * W + lane];
      const R from_lo = dpp_move<0x138>(Bv), from_hi = dpp_move<0x130>(Bv);
      R sh = a > 0 ? from_hi : from_lo;                                       // Bv[lane + a]
      if ((unsigned(lane + a) >= unsigned(W)) | !valid) sh = rinf<R>();
      // inf + finite and inf + inf stay inf
      R pm1, pe1, pm0, pe0;
      seg_softmin_parts<W, R>(Fl + lamL[l] + sh, pm1, pe1);
      seg_softmin_parts<W, R>(Fl + Bv, pm0, pe0);
      if (lane == l) {
        m1 = pm1;
        e1 = pe1;
        m0 = pm0;
        e0 = pe0;
      }
      Bv = smin2u<R>(Bv, sh + lamL[l]);
      if (!valid) Bv = rinf<R>();
    }
    const R my1 = m1 - SoftUnits<R>::L(e1);
    const R myM = (my1 - (m0 - SoftUnits<R>::L(e0))) * unit;
    // soft row value B_0(0) sits on lane N
    const R rowv = __shfl(Bv, N, W);
    if (lane < n) {
      if (MODE == MODE_UPDATE) write_out<R>(out, w, mylam - omega * myM);
      if (MODE == MODE_EVAL) write_out<R>(out, w, SoftUnits<R>::E(rowv - my1));
    }
    if (lane == 0) rowpart = double(rowv * unit);
  }
  double part = block_sum(rowpart, red);
  store_partial(part, A.partial, item);
}

// ---------------------------------------------------------------- long rows (exactly one)
template <typename R>
struct MinState {   // hard: (m, a, m2); soft adds s = sum_{k != a} exp(-(lam_k - m2)/T)
  R m, m2, s;
  int32_t a;
};

template <typename R, bool SOFT>
__device__ inline MinState<R> ms_combine(MinState<R> x, MinState<R> y, R T) {
  if (y.m < x.m || (y.m == x.m && y.a < x.a)) {
    MinState<R> t = x;
    x = y;
    y = t;
  }
  MinState<R> r;
  r.m = x.m;
  r.a = x.a;
  r.m2 = x.m2 < y.m ? x.m2 : y.m;
  r.s = R(0);
  if (SOFT && r.m2 != rinf<R>()) {
    R sx = (x.m2 == rinf<R>()) ? R(0) : x.s * r_exp<R>(-(x.m2 - r.m2) / T);
    R ys = (y.m2 == rinf<R>()) ? R(0) : y.s * r_exp<R>(-(y.m2 - y.m) / T);
    R sy = (y.m == rinf<R>()) ? R(0) : (R(1) + ys) * r_exp<R>(-(y.m - r.m2) / T);
    r.s = sx + sy;
  }
  return r;
}

template <typename R, bool SOFT>
__device__ inline MinState<R> ms_shfl_xor(MinState<R> v, int off) {
  MinState<R> o;
  o.m = __shfl_xor(v.m, off);
  o.m2 = __shfl_xor(v.m2, off);
  o.s = SOFT ? __shfl_xor(v.s, off) : R(0);
  o.a = __shfl_xor(v.a, off);
  return o;
}

// one wave per projection row (four rows per block), or for long rows one
// block per row (long_wpr = 4); each lane keeps up to LONG_REG of its row's
// multipliers in registers between the two passes
constexpr int LONG_REG = 8;
constexpr int32_t LONG_GROUP = 8;   // consecutive projection-row blocks per XCD turn

// LONG_BATCH: record loads in flight per lane
template <typename R, bool SOFT, int MODE, int LONG_BATCH>
__device__ void long_rows(const SweepArgs& A, const R* __restrict__ rin, R* __restrict__ out, R omega, R T,
                          R gam, double* red, int32_t item) {
  __shared__ R xm[4], xm2[4], xs[4];
  __shared__ int32_t xa[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wpr = A.long_wpr;   // uniform
  const int sub = wave & (wpr - 1);
  const int32_t lr = (item - A.n_short_blocks) * (4 / wpr) + wave / wpr;
  const bool has = lr < A.n_long;
  const int32_t j = has ? A.n_short + A.long_perm[lr] : 0;
  const int32_t step = 64 * wpr, i0 = sub * 64 + lane;
  const int32_t s = has ? A.rrow_ptr[j] : 0;
  const int32_t n = has ? A.rrow_ptr[j + 1] - s : 0;
  MinState<R> st;
  st.m = rinf<R>();
  st.m2 = rinf<R>();
  st.s = R(0);
  st.a = INT32_MAX;
  // The first LONG_REG entries of every lane are loaded without branches
  // (past the row's end a lane loads the row's first entry and ignores it), so
  // that all loads of a batch are in flight together: the words, then the
  // records in batches of LONG_BATCH.
  uint32_t wv[LONG_REG];
  R lv[LONG_REG];
#pragma unroll
  for (int u = 0; u < LONG_REG; ++u) {
    const int32_t i = i0 + step * u;
    wv[u] = n > 0 ? A.word[s + (i < n ? i : 0)] : 0u;
  }
#pragma unroll
  for (int u0 = 0; u0 < LONG_REG; u0 += LONG_BATCH) {
    if (sub * 64 + step * u0 >= n) break;   // uniform: no lane of the wave has entries left
    RecRaw<R> raw[LONG_BATCH];
#pragma unroll
    for (int u = 0; u < LONG_BATCH; ++u) raw[u].load(rin, wv[u0 + u] & W_VAR_MASK);
    R dv[LONG_BATCH];
    if (A.dir)
#pragma unroll
      for (int u = 0; u < LONG_BATCH; ++u) dv[u] = static_cast<const R*>(A.dir)[slot_index(A, wv[u0 + u])];
#pragma unroll
    for (int u = 0; u < LONG_BATCH; ++u) {
      const int32_t i = i0 + step * (u0 + u);
      R v = raw[u].lambda(int((wv[u0 + u] >> W_SLOT_SHIFT) & 7u));
      if (A.dir) v += gam * dv[u];
      lv[u0 + u] = v;
      if (i < n) {
        MinState<R> one;
        one.m = v;
        one.m2 = rinf<R>();
        one.s = R(0);
        one.a = i;
        st = ms_combine<R, SOFT>(st, one, T);
      }
    }
  }
  for (int32_t i = i0 + step * LONG_REG; i < n; i += step) {   // rows longer than step * LONG_REG
    MinState<R> one;
    one.m = row_lambda<R>(A, rin, A.word[s + i], gam);
    one.m2 = rinf<R>();
    one.s = R(0);
    one.a = i;
    st = ms_combine<R, SOFT>(st, one, T);
  }
  for (int off = 32; off > 0; off >>= 1) st = ms_combine<R, SOFT>(st, ms_shfl_xor<R, SOFT>(st, off), T);
  if (wpr > 1) {
    // the row's waves combine their states in index order: every wave of
    // the row ends with the same state
    if (lane == 0) {
      xm[wave] = st.m;
      xm2[wave] = st.m2;
      xs[wave] = st.s;
      xa[wave] = st.a;
    }
    __syncthreads();
    const int w0 = wave & ~(wpr - 1);
    MinState<R> acc;
    acc.m = xm[w0];
    acc.m2 = xm2[w0];
    acc.s = xs[w0];
    acc.a = xa[w0];
    for (int q = 1; q < wpr; ++q) {
      MinState<R> o;
      o.m = xm[w0 + q];
      o.m2 = xm2[w0 + q];
      o.s = xs[w0 + q];
      o.a = xa[w0 + q];
      acc = ms_combine<R, SOFT>(acc, o, T);
    }
    st = acc;
  }
  double rowpart = 0.0;
  if (has) {
    R rowv = st.m;
    R tot = R(0);
    if (SOFT) {
      tot = (st.m2 == rinf<R>()) ? R(0) : st.s * r_exp<R>(-(st.m2 - st.m) / T);
      rowv = st.m - T * r_log<R>(R(1) + tot);
    }
    if (MODE != MODE_BOUND) {
      auto finish = [&](int32_t i, uint32_t w, R lam) {
        R M, mu = R(0);
        if (!SOFT) {
          M = lam - (i == st.a ? st.m2 : st.m);
        } else {
          R others;
          if (i == st.a) {
            others = st.m2 - T * r_log<R>(st.s);
          } else {
            R e = r_exp<R>(-(lam - st.m) / T);
            others = st.m - T * r_log<R>((R(1) + tot) - e);
          }
          M = lam - others;
          mu = r_exp<R>(-(lam - rowv) / T);
        }
        if (MODE == MODE_UPDATE) write_out<R>(out, w, lam - omega * M);
        if (MODE == MODE_EVAL) write_out<R>(out, w, SOFT ? mu : M);
        if (MODE == MODE_SUBGRAD)
          A.gsub[slot_index(A, w)] = uint8_t(i == st.a ? 1 : 0);
      };
#pragma unroll
      for (int u = 0; u < LONG_REG; ++u) {
        const int32_t i = i0 + step * u;
        if (i < n) finish(i, wv[u], lv[u]);
      }
      for (int32_t i = i0 + step * LONG_REG; i < n; i += step) {
        const uint32_t w = A.word[s + i];
        finish(i, w, row_lambda<R>(A, rin, w, gam));
      }
    }
    if (lane == 0 && sub == 0) rowpart = double(rowv);
  }
  double part = block_sum(rowpart, red);
  store_partial(part, A.partial, item);
}

template <typename R, bool SOFT>
constexpr size_t smem_bytes() {
  return SOFT ? (SOFT_FTAB + 256) * sizeof(R) + 256 : 768 * sizeof(R);
}

// TB > 0: the hard form's launch has one-lane-per-row tiles, whose record
// loads go TB at a time (their register use sets the occupancy of the whole
// kernel, so launches without tiles take the instantiation TB = 0)
template <typename R, bool SOFT, int MODE, int TB>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs A, const R* __restrict__ rin, R* __restrict__ out,
                                               R omega, R T) {
  __shared__ __align__(16) unsigned char smem[smem_bytes<R, SOFT>()];
  __shared__ double red[256];
  if (A.skip && *A.skip) return;   // uniform across the grid
  if (blockIdx.x == 0 && A.prev_partial) reduce_partials(A.prev_partial, A.prev_n, A.prev_offset, A.prev_out, red);
  const R gam = A.gamma ? R(*A.gamma) : R(0);
  // Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
  // The hard form takes the item of block b from the per-XCD table of the
  // sweep layout (region b % 8, in key order).  The smoothed form gives each
  // XCD a contiguous range of short-row blocks and projection-row blocks in
  // groups of LONG_GROUP consecutive blocks, group g on XCD g % 8, the heavier
  // projection-row blocks first.
  const int32_t x = int32_t(blockIdx.x % 8u), k0 = int32_t(blockIdx.x / 8u);
  if (!SOFT) {
    if (k0 >= A.xcd_stride) return;
    const int32_t item = A.xcd_item[x * A.xcd_stride + k0];
    if (item < 0) return;
    if constexpr (TB > 0) {
      if (item < A.n_tile_items) {
        tile_block<R, MODE, TB>(A, rin, out, omega, gam, red, item);
        return;
      }
    }
    if (item < A.n_short_blocks) short_wave_hard<R, MODE>(A, rin, out, omega, gam, smem, red, item);
    else long_rows<R, false, MODE, (TB > 0 ? 4 : 2)>(A, rin, out, omega, T, gam, red, item);
    return;
  }
  int32_t item;
  {
    const int32_t n_long_blocks = A.n_items - A.n_short_blocks;
    const int32_t lx = (n_long_blocks + 8 * LONG_GROUP - 1) / (8 * LONG_GROUP) * LONG_GROUP;
    if (k0 < lx) {
      const int32_t li = ((k0 / LONG_GROUP) * 8 + x) * LONG_GROUP + k0 % LONG_GROUP;
      if (li >= n_long_blocks) return;
      item = A.n_short_blocks + li;
    } else {
      const int32_t pc = (A.n_short_blocks + 7) / 8;
      const int32_t c = x * pc + (k0 - lx);
      if (k0 - lx >= pc || c >= A.n_short_blocks) return;
      item = c;
    }
  }
  if (item < A.n_short_blocks) {
    const int32_t nb8 = (A.soft_c8 + soft_rpb<8>() - 1) / soft_rpb<8>();
    const int32_t nb16 = (A.soft_c16 + soft_rpb<16>() - 1) / soft_rpb<16>();
    const int32_t c816 = A.soft_c8 + A.soft_c16;
    if (item < nb8)
      short_rows_soft<R, MODE, 8>(A, rin, out, omega, T, smem, red, item, item, 0, A.soft_c8);
    else if (item < nb8 + nb16)
      short_rows_soft<R, MODE, 16>(A, rin, out, omega, T, smem, red, item, item - nb8, A.soft_c8, c816);
    else
      short_rows_soft<R, MODE, 32>(A, rin, out, omega, T, smem, red, item, item - nb8 - nb16, c816,
                                   A.n_short);
  } else {
    long_rows<R, true, MODE, 2>(A, rin, out, omega, T, gam, red, item);
  }
}

// ---------------------------------------------------------------- state import / export
template <typename R>
__global__ void k_import(const R* lam, const uint32_t* word, int64_t nnz, R* rec) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) write_out<R>(rec, word[e], lam[e]);
}

template <typename R>
__global__ void k_set_cost(const int32_t* free_var, const double* c64, const uint8_t* deg, int64_t nfree, R* rec0,
                           R* rec1) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  const R c = R(c64[free_var[i]]), rd = R(1) / R(deg[i]);
  rec0[size_t(i) * REC + REC_COST] = c;
  rec0[size_t(i) * REC + REC_RDEG] = rd;
  if (rec1) {
    rec1[size_t(i) * REC + REC_COST] = c;
    rec1[size_t(i) * REC + REC_RDEG] = rd;
  }
}

template <typename R>
__global__ void k_export(const R* rec, const uint32_t* word, int64_t nnz, R* lam) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) lam[e] = cur_lambda<R>(rec, word[e]);
}

template <typename R>
__global__ void k_init_lambda(const uint32_t* word, const int32_t* free_var, const double* c64, const uint8_t* deg,
                              int64_t nnz, R* lam) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t i = word[e] & W_VAR_MASK;
  const R c = R(c64[free_var[i]]);
  lam[e] = c / R(deg[i]);
}

__global__ void k_write_offset(double* out, double v) { *out = v; }

__global__ __launch_bounds__(256) void k_reduce_last(const double* partial, int n, double offset, double* out) {
  __shared__ double red[256];
  reduce_partials(partial, n, offset, out, red);
}

// one sweep launch; with timing events the launch records the kernel's own
// start and end (hipExtLaunchKernelGGL), as a kernel trace does
template <typename R, bool SOFT, int MODE, int TB = 0>
void launch_sweep(hipStream_t st, unsigned grid, hipEvent_t e0, hipEvent_t e1, const SweepArgs& A, const R* ri,
                  R* ro, R omega, R T) {
  if (e0)
    hipExtLaunchKernelGGL(k_sweep<R, SOFT, MODE, TB>, dim3(grid), dim3(256), 0, st, e0, e1, 0, A, ri, ro, omega, T);
  else
    k_sweep<R, SOFT, MODE, TB><<<grid, 256, 0, st>>>(A, ri, ro, omega, T);
}

// Tile record loads: 16 in flight per lane once there are at least
// TILE_WIDE_BATCH tiles (more latency hidden per wave, 1000-face pair 46 ->
// 42 us), 8 below (the 500-face pair's 900 tiles are 1 % faster so); FP64
// sweeps take one instantiation (their batches are two records).
constexpr int32_t TILE_WIDE_BATCH = 2048;
template <typename R, int MODE>
void launch_hard(int32_t n_tiles, hipStream_t st, unsigned grid, hipEvent_t e0, hipEvent_t e1, const SweepArgs& A,
                 const R* ri, R* ro, R omega, R T) {
  if (n_tiles <= 0) launch_sweep<R, false, MODE, 0>(st, grid, e0, e1, A, ri, ro, omega, T);
  else if (sizeof(R) == 4 && n_tiles >= TILE_WIDE_BATCH)
    launch_sweep<R, false, MODE, 16>(st, grid, e0, e1, A, ri, ro, omega, T);
  else launch_sweep<R, false, MODE, 8>(st, grid, e0, e1, A, ri, ro, omega, T);
}

}  // namespace

// ============================================================================
// host side (shared with rounding and the backward pass)
// ============================================================================
// per-launch partials of one sweep (hard and smoothed forms): the partial
// buffer holds two halves of this many doubles
static int64_t sweep_partial_cap(const dm_ctx* ctx) {
  const int64_t c32 = ctx->n_short - ctx->soft_c8 - ctx->soft_c16;
  const int64_t soft_blocks = (ctx->soft_c8 + soft_rpb<8>() - 1) / soft_rpb<8>() +
                              (ctx->soft_c16 + soft_rpb<16>() - 1) / soft_rpb<16>() +
                              (c32 + soft_rpb<32>() - 1) / soft_rpb<32>();
  return std::max<int64_t>(int64_t(ctx->n_tile_items) + (ctx->n_chunks + 3) / 4, soft_blocks) +
         ctx->n_long_items;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

SolverLayout solver_layout(const dm_ctx* ctx, size_t real_bytes) {
  SolverLayout L;
  L.rec_bytes = align256(size_t(std::max<int64_t>(ctx->n_free, 1)) * REC * real_bytes);
  L.part_off = 2 * L.rec_bytes;
  L.part_count = size_t(2 * std::max<int64_t>(sweep_partial_cap(ctx), 1));
  L.total = L.part_off + align256(L.part_count * sizeof(double));
  return L;
}

// the caller's workspace of this precision, checked against the current
// problem (NULL when none is attached)
static dm_status solver_workspace(dm_ctx* ctx, size_t real_bytes, unsigned char** base, SolverLayout* L) {
  const int k = real_bytes == 4 ? 0 : 1;
  *base = static_cast<unsigned char*>(ctx->ws_ptr[k]);
  *L = solver_layout(ctx, real_bytes);
  if (*base && ctx->ws_bytes[k] < L->total)
    return dm_fail(ctx, DM_ERR_WORKSPACE, "the attached %s solver workspace has %zu bytes; the current problem needs %zu",
                   k == 0 ? "FP32" : "FP64", ctx->ws_bytes[k], L->total);
  return DM_OK;
}

template <typename R>
dm_status dual_import(dm_ctx* ctx, const R* lam, DArr<unsigned char>* bufs) {
  const size_t bytes = size_t(std::max<int64_t>(ctx->n_free, 1)) * REC * sizeof(R);
  unsigned char* ws = nullptr;
  SolverLayout L;
  if (bufs == ctx->rec) DM_TRY(solver_workspace(ctx, sizeof(R), &ws, &L));
  if (ws) {   // the solver's records live in the caller's workspace
    bufs[0].attach(ws, bytes);
    bufs[1].attach(ws + L.rec_bytes, bytes);
  } else {
    DM_ALLOC(ctx, bufs[0], bytes);
    DM_ALLOC(ctx, bufs[1], bytes);
  }
  DM_HIP(ctx, hipMemsetAsync(bufs[0].p, 0, bytes, ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(bufs[1].p, 0, bytes, ctx->stream));
  R* r0 = reinterpret_cast<R*>(bufs[0].p);
  R* r1 = reinterpret_cast<R*>(bufs[1].p);
  if (ctx->n_free > 0)
    k_set_cost<R><<<grid_for(ctx->n_free, 256), 256, 0, ctx->stream>>>(ctx->free_var.p, ctx->cost64.p,
                                                                       ctx->var_deg.p, ctx->n_free, r0, r1);
  if (ctx->nnz > 0)
    k_import<R><<<grid_for(ctx->nnz, 256), 256, 0, ctx->stream>>>(lam, ctx->rent_word.p, ctx->nnz, r0);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

template <typename R>
dm_status dual_export(dm_ctx* ctx, const unsigned char* rec, R* lam) {
  if (ctx->nnz > 0)
    k_export<R><<<grid_for(ctx->nnz, 256), 256, 0, ctx->stream>>>(reinterpret_cast<const R*>(rec),
                                                                  ctx->rent_word.p, ctx->nnz, lam);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

// one sweep over all rows; mode 0 update rec_in -> out, 1 write M (or mu) to
// out per slot, 2 bound only; the bound goes to *bound_out (device)
template <typename R>
dm_status dual_sweep(dm_ctx* ctx, int mode, bool soft, const unsigned char* rin, unsigned char* out, R omega,
                     R T, double* bound_out, const SweepExt* ext) {
  if (soft && (ext || mode == MODE_SUBGRAD))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "direction, skip and subgradient sweeps use the hard minimum");
  if (soft && ctx->max_short > SOFT_MAX_ROW)
    return dm_fail(ctx, DM_ERR_WORKSPACE, "smoothed rows support at most %d entries (found %d)", SOFT_MAX_ROW,
                   ctx->max_short);
  SweepArgs A;
  A.word = ctx->rent_word.p;
  A.rrow_ptr = ctx->rrow_ptr.p;
  A.rrow_b = ctx->rrow_b.p;
  A.chunk_desc = ctx->chunk_desc.p;
  A.chunk_mask = ctx->chunk_mask.p;
  A.chunk_word = ctx->chunk_word.p;
  A.chunk_b = ctx->chunk_b.p;
  A.n_chunks = ctx->n_chunks;
  A.soft_row = ctx->soft_row.p;
  A.soft_c8 = int32_t(ctx->soft_c8);
  A.soft_c16 = int32_t(ctx->soft_c16);
  const int64_t c32 = ctx->n_short - ctx->soft_c8 - ctx->soft_c16;
  const int64_t soft_blocks = (ctx->soft_c8 + soft_rpb<8>() - 1) / soft_rpb<8>() +
                              (ctx->soft_c16 + soft_rpb<16>() - 1) / soft_rpb<16>() +
                              (c32 + soft_rpb<32>() - 1) / soft_rpb<32>();
  A.n_tile_items = soft ? 0 : ctx->n_tile_items;
  A.n_tiles = ctx->n_tiles;
  A.tile_word = ctx->tile_word.p;
  A.n_short_blocks = soft ? int32_t(soft_blocks) : ctx->n_tile_items + int32_t((ctx->n_chunks + 3) / 4);
  // projection rows: a wave each, or a whole block each when they are long
  const int64_t n_long = ctx->n_rows - ctx->n_short;
  A.long_wpr = ctx->long_wpr;
  A.n_long = int32_t(n_long);
  A.long_perm = ctx->long_perm.p;
  A.xcd_item = ctx->xcd_item.p;
  A.xcd_stride = ctx->xcd_stride;
  const int64_t n_long_blocks = ctx->n_long_items;
  A.n_short = int32_t(ctx->n_short);
  A.n_rows = int32_t(ctx->n_rows);
  A.plane = ctx->n_free;
  A.dir = ext ? ext->dir : nullptr;
  A.gamma = ext ? ext->gamma : nullptr;
  A.skip = ext ? ext->skip : nullptr;
  A.gsub = ext ? ext->gsub : nullptr;
  const int64_t nblocks = int64_t(A.n_short_blocks) + n_long_blocks;
  if (nblocks == 0) {
    DM_TRY(dual_flush(ctx));
    if (bound_out) k_write_offset<<<1, 1, 0, ctx->stream>>>(bound_out, ctx->offset);
    DM_LAUNCH_CHECK(ctx);
    return DM_OK;
  }
  // two halves of the partial buffer alternate between consecutive launches;
  // with a caller workspace of this precision they live there
  const int64_t cap = sweep_partial_cap(ctx);
  unsigned char* ws = nullptr;
  SolverLayout L;
  DM_TRY(solver_workspace(ctx, sizeof(R), &ws, &L));
  if (ws) {
    double* want = reinterpret_cast<double*>(ws + L.part_off);
    if (ctx->partial.p != want || ctx->partial.n < size_t(2 * cap)) {
      DM_TRY(dual_flush(ctx));
      ctx->partial.attach(want, L.part_count);
    }
  } else if (ctx->partial.view || ctx->partial.n < size_t(2 * cap)) {
    DM_TRY(dual_flush(ctx));
    DM_ALLOC(ctx, ctx->partial, size_t(2 * cap));
  }
  double* mine = ctx->partial.p + (ctx->pend_half ^ 1) * cap;
  A.partial = mine;
  A.prev_partial = ctx->pend_out ? ctx->pend_partial : nullptr;
  A.prev_n = ctx->pend_n;
  A.prev_offset = ctx->pend_offset;
  A.prev_out = ctx->pend_out;
  const R* ri = reinterpret_cast<const R*>(rin);
  R* ro = reinterpret_cast<R*>(out);
  A.n_items = int32_t(nblocks);
  // 8 XCDs x blocks per XCD, see k_sweep
  const int64_t long_slots = (n_long_blocks + 8 * LONG_GROUP - 1) / (8 * LONG_GROUP) * LONG_GROUP;
  const unsigned grid = soft ? unsigned(8 * (long_slots + (A.n_short_blocks + 7) / 8))
                             : unsigned(8 * int64_t(ctx->xcd_stride));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
      hipEvent_t e;
      DM_HIP(ctx, hipEventCreate(&e));
      ctx->ev_pool.push_back(e);
    }
    e0 = ctx->ev_pool[ctx->ev_used];
    e1 = ctx->ev_pool[ctx->ev_used + 1];
    ctx->ev_used += 2;
  }
  hipStream_t st = ctx->stream;
  if (soft) {
    if (mode == MODE_UPDATE) launch_sweep<R, true, MODE_UPDATE>(st, grid, e0, e1, A, ri, ro, omega, T);
    else if (mode == MODE_EVAL) launch_sweep<R, true, MODE_EVAL>(st, grid, e0, e1, A, ri, ro, omega, T);
    else launch_sweep<R, true, MODE_BOUND>(st, grid, e0, e1, A, ri, ro, omega, T);
  } else {
    const int32_t tiles = ctx->n_tiles;
    if (mode == MODE_UPDATE) launch_hard<R, MODE_UPDATE>(tiles, st, grid, e0, e1, A, ri, ro, omega, T);
    else if (mode == MODE_EVAL) launch_hard<R, MODE_EVAL>(tiles, st, grid, e0, e1, A, ri, ro, omega, T);
    else if (mode == MODE_BOUND) launch_hard<R, MODE_BOUND>(tiles, st, grid, e0, e1, A, ri, ro, omega, T);
    else launch_hard<R, MODE_SUBGRAD>(tiles, st, grid, e0, e1, A, ri, ro, omega, T);
  }
  DM_LAUNCH_CHECK(ctx);
  ctx->pend_half ^= 1;
  ctx->pend_partial = mine;
  ctx->pend_n = int32_t(nblocks);
  ctx->pend_offset = ctx->offset;
  ctx->pend_out = bound_out;
  return DM_OK;
}

// sum the partials of the last launch whose bound has not been written yet
dm_status dual_flush(dm_ctx* ctx) {
  if (ctx->pend_out) {
    k_reduce_last<<<1, 256, 0, ctx->stream>>>(ctx->pend_partial, ctx->pend_n, ctx->pend_offset, ctx->pend_out);
    DM_LAUNCH_CHECK(ctx);
  }
  ctx->pend_out = nullptr;
  return DM_OK;
}

extern "C" dm_status dm_timing_enable(dm_ctx* ctx, int32_t enable) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return DM_OK;
}

extern "C" dm_status dm_timing_read(dm_ctx* ctx, int64_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return DM_ERR_INVALID_ARG;
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.0f;
    DM_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
    tot += ms;
  }
  *launches = int64_t(ctx->ev_used / 2);
  *total_ms = tot;
  ctx->ev_used = 0;
  return DM_OK;
}

template dm_status dual_import<float>(dm_ctx*, const float*, DArr<unsigned char>*);
template dm_status dual_import<double>(dm_ctx*, const double*, DArr<unsigned char>*);
template dm_status dual_export<float>(dm_ctx*, const unsigned char*, float*);
template dm_status dual_export<double>(dm_ctx*, const unsigned char*, double*);
template dm_status dual_sweep<float>(dm_ctx*, int, bool, const unsigned char*, unsigned char*, float, float, double*,
                                     const SweepExt*);
template dm_status dual_sweep<double>(dm_ctx*, int, bool, const unsigned char*, unsigned char*, double, double,
                                      double*, const SweepExt*);

static dm_status check_solver(dm_ctx* ctx, int32_t msg_prec) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "no product space built");
  if (!ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "no costs built");
  if (msg_prec != DM_PREC_FP32 && msg_prec != DM_PREC_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "message precision must be FP32 or FP64");
  return DM_OK;
}

template <typename R>
static dm_status solve_impl(dm_ctx* ctx, int32_t iters, R omega, R T, R* lam, double* trace) {
  DM_TRY(dual_import<R>(ctx, lam, ctx->rec));
  const bool soft = T > R(0);
  for (int32_t t = 0; t < iters; ++t)
    DM_TRY(dual_sweep<R>(ctx, MODE_UPDATE, soft, ctx->rec[t & 1].p, ctx->rec[(t + 1) & 1].p, omega, T,
                         trace ? trace + t : nullptr));
  DM_TRY(dual_flush(ctx));
  DM_TRY(dual_export<R>(ctx, ctx->rec[iters & 1].p, lam));
  return DM_OK;
}

extern "C" dm_status dm_dual_solve(dm_ctx* ctx, int32_t iters, double omega, double temperature,
                                   int32_t msg_prec, void* lambda, double* lb_trace) {
  DM_TRY(check_solver(ctx, msg_prec));
  ctx->err.clear();
  if (iters < 0 || (!lambda && ctx->nnz > 0))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_dual_solve: bad arguments");
  if (!(omega > 0.0 && omega <= 1.0)) return dm_fail(ctx, DM_ERR_INVALID_ARG, "omega must be in (0, 1]");
  if (!(temperature >= 0.0)) return dm_fail(ctx, DM_ERR_INVALID_ARG, "temperature must be >= 0");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return solve_impl<float>(ctx, iters, float(omega), float(temperature), static_cast<float*>(lambda), lb_trace);
  return solve_impl<double>(ctx, iters, omega, temperature, static_cast<double*>(lambda), lb_trace);
}

extern "C" dm_status dm_init_lambda(dm_ctx* ctx, int32_t msg_prec, void* lambda) {
  DM_TRY(check_solver(ctx, msg_prec));
  if (!lambda && ctx->nnz > 0) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_init_lambda: NULL lambda");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (ctx->nnz == 0) return DM_OK;
  if (msg_prec == DM_PREC_FP32)
    k_init_lambda<float><<<grid_for(ctx->nnz, 256), 256, 0, ctx->stream>>>(
        ctx->rent_word.p, ctx->free_var.p, ctx->cost64.p, ctx->var_deg.p, ctx->nnz, static_cast<float*>(lambda));
  else
    k_init_lambda<double><<<grid_for(ctx->nnz, 256), 256, 0, ctx->stream>>>(
        ctx->rent_word.p, ctx->free_var.p, ctx->cost64.p, ctx->var_deg.p, ctx->nnz, static_cast<double*>(lambda));
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

template <typename R>
static dm_status bound_impl(dm_ctx* ctx, const R* lam, R T, double* out) {
  DArr<unsigned char> bufs[2];
  DM_TRY(dual_import<R>(ctx, lam, bufs));
  DM_ALLOC(ctx, ctx->scal, 16);
  DM_TRY(dual_sweep<R>(ctx, MODE_BOUND, T > R(0), bufs[0].p, nullptr, R(0), T, ctx->scal.p));
  DM_TRY(dual_flush(ctx));
  DM_HIP(ctx, hipMemcpyAsync(out, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DM_OK;
}

extern "C" dm_status dm_lower_bound(dm_ctx* ctx, const void* lambda, double temperature, int32_t msg_prec,
                                    double* lb) {
  DM_TRY(check_solver(ctx, msg_prec));
  if ((!lambda && ctx->nnz > 0) || !lb) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_lower_bound: NULL argument");
  if (!(temperature >= 0.0)) return dm_fail(ctx, DM_ERR_INVALID_ARG, "temperature must be >= 0");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return bound_impl<float>(ctx, static_cast<const float*>(lambda), float(temperature), lb);
  return bound_impl<double>(ctx, static_cast<const double*>(lambda), temperature, lb);
}

extern "C" dm_status dm_workspace_query(const dm_ctx* ctx, int32_t stage, size_t* bytes) {
  if (!ctx || !bytes) return DM_ERR_INVALID_ARG;
  if (stage != DM_WS_SOLVE_FP32 && stage != DM_WS_SOLVE_FP64) return DM_ERR_INVALID_ARG;
  if (!ctx->has_space) return DM_ERR_STATE;
  *bytes = solver_layout(ctx, stage == DM_WS_SOLVE_FP32 ? 4 : 8).total;
  return DM_OK;
}

extern "C" dm_status dm_set_workspace(dm_ctx* ctx, int32_t stage, void* ptr, size_t bytes) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (stage != DM_WS_SOLVE_FP32 && stage != DM_WS_SOLVE_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_set_workspace: unknown stage %d", stage);
  const int k = stage == DM_WS_SOLVE_FP32 ? 0 : 1;
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));   // a pending bound may still read the old partials
  if (ptr) {
    if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
      return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_set_workspace: the buffer must be 256-byte aligned");
    if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "dm_set_workspace: no problem built");
    const size_t need = solver_layout(ctx, k == 0 ? 4 : 8).total;
    if (bytes < need)
      return dm_fail(ctx, DM_ERR_WORKSPACE, "dm_set_workspace: %zu bytes given, %zu needed", bytes, need);
  }
  // the solver's state moves: its own arrays (or views of the old buffer) go
  ctx->rec[0].release();
  ctx->rec[1].release();
  ctx->partial.release();
  ctx->ws_ptr[k] = ptr;
  ctx->ws_bytes[k] = ptr ? bytes : 0;
  return DM_OK;
}
