// Launch layout of the row sweep (the row-parallel min-marginal sweep of
// Sec. 3.2 / Eq. (D), mapped onto the eight XCDs of the chip).
//
// Each XCD has its own L2, and a multiplier record that rows on several XCDs
// read and write is fetched, and written back as a partial line, once per
// XCD.  The layout therefore gives every XCD a spatial region of the problem:
//   * every free variable gets a key, the rank of its X element's owner face
//     in the Morton order of the X face centroids (a face owns itself; an
//     edge or a vertex is owned by its adjacent face of lowest rank).  A
//     generic problem without meshes keys a variable by its index;
//   * the keys are cut into eight contiguous ranges of equal entry counts,
//     the regions; a short row and an X projection row take the smallest key
//     of their entries, so they land in the region that owns (nearly) all of
//     their variables.  Y projection rows span every region and are dealt to
//     the regions in turn, spread evenly over each region's key range;
//   * short rows are packed into wave chunks in key order, projection rows
//     are ordered by region and key, and block b of a launch runs on XCD
//     b % 8 (the order in which workgroups are dealt to the XCDs), taking
//     the items of region b % 8 in key order from a per-XCD table, so that
//     rows that share variables run on one XCD at nearly the same time.
// Only the launch order changes: the reduced problem's rows, entries and
// record slots are untouched, and every row is still swept exactly once.
#include <algorithm>
#include <climits>

#include "dm_internal.h"

namespace {

constexpr int NREG = 8;           // XCDs
constexpr int PACK_SEG = 4096;    // entries per segment of the parallel chunk packing

// ---------------------------------------------------------------- keys
// bounding box of the vertices: out[0..2] minimum, out[3..5] maximum
__global__ __launch_bounds__(256) void k_bbox(const float* v, int32_t nv, float* out) {
  __shared__ float sh[6][256];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = threadIdx.x; i < nv; i += 256)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], v[3 * i + k]);
      hi[k] = fmaxf(hi[k], v[3 * i + k]);
    }
  for (int k = 0; k < 3; ++k) {
    sh[k][threadIdx.x] = lo[k];
    sh[3 + k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o)
      for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = fminf(sh[k][threadIdx.x], sh[k][threadIdx.x + o]);
        sh[3 + k][threadIdx.x] = fmaxf(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[threadIdx.x] = sh[threadIdx.x][0];
}

__device__ inline uint32_t spread3(uint32_t x) {   // 10 bits -> every third bit of 30
  x &= 0x3FFu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// 30-bit Morton code of every face centroid on a 1024^3 grid over the box
__global__ void k_face_morton(const float* v, const int32_t* f, int32_t nf, const float* box, uint32_t* key,
                              int32_t* val) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    const float c = (v[3 * f[3 * i] + k] + v[3 * f[3 * i + 1] + k] + v[3 * f[3 * i + 2] + k]) * (1.0f / 3.0f);
    const float ext = box[3 + k] - box[k];
    const float u = ext > 0.0f ? (c - box[k]) / ext : 0.0f;
    q[k] = uint32_t(fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f));
  }
  key[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  val[i] = i;
}

__global__ void k_rank_of(const int32_t* order, int32_t n, int32_t* rank) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) rank[order[i]] = i;
}

// owner rank of every edge and vertex: the lowest rank of an adjacent face
__global__ void k_elem_rank(const int32_t* faces, const int32_t* face_edge, const int32_t* frank, int32_t nf,
                            int32_t* erank, int32_t* vrank) {
  const int32_t f = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int32_t r = frank[f];
  for (int k = 0; k < 3; ++k) {
    atomicMin(&erank[face_edge[3 * f + k]], r);
    atomicMin(&vrank[faces[3 * f + k]], r);
  }
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// empty key ranges of the NREG regions: (INT32_MAX, -1) pairs, one launch
__global__ void k_bounds_init(int32_t* bounds) {
  const int t = int(threadIdx.x);
  if (t < 2 * NREG) bounds[t] = (t & 1) ? -1 : INT32_MAX;
}

// key of every free variable: the rank of its X element's owner face
__global__ void k_var_key_mesh(const int32_t* free_var, const int32_t* code, const int32_t* frank,
                               const int32_t* erank, const int32_t* vrank, int64_t n, int32_t* vkey) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = free_var[i];
  const int32_t cls = code[4 * p], id = code[4 * p + 1];
  vkey[i] = cls == 0 ? frank[id] : (cls == 1 ? erank[id] : vrank[id]);
}

__global__ void k_iota(int32_t* a, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = int32_t(i);
}

// entries per key: every free variable adds its row count to its key's bin.
// Each block takes a contiguous range of variables (in canonical order, so
// few distinct keys) into an LDS histogram and adds its non-empty bins to
// the global one; nkeys <= KEY_BINS_LDS.
constexpr int KEY_BINS_LDS = 16384;
constexpr int KEY_VARS_PER_BLOCK = 4096;

__global__ __launch_bounds__(256) void k_key_weight(const int32_t* vkey, const uint8_t* deg, int64_t nfree,
                                                    int32_t nkeys, int32_t* w) {
  extern __shared__ int32_t hist[];
  for (int32_t k = threadIdx.x; k < nkeys; k += 256) hist[k] = 0;
  __syncthreads();
  const int64_t lo = int64_t(blockIdx.x) * KEY_VARS_PER_BLOCK;
  const int64_t hi = lo + KEY_VARS_PER_BLOCK < nfree ? lo + KEY_VARS_PER_BLOCK : nfree;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) atomicAdd(&hist[vkey[i]], int32_t(deg[i]));
  __syncthreads();
  for (int32_t k = threadIdx.x; k < nkeys; k += 256)
    if (hist[k]) atomicAdd(&w[k], hist[k]);
}

// a generic problem keys every variable by itself: its weight is its row count
__global__ void k_deg_weight(const uint8_t* deg, int64_t n, int32_t* w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = deg[i];
}

// region of a key: the eighth of all entries in which the middle of the
// key's own entries falls
__device__ inline int32_t region_of(const int32_t* pre, const int32_t* w, int32_t k, int64_t total) {
  const int64_t mid2 = 2 * int64_t(pre[k]) + w[k];
  const int64_t r = total > 0 ? (NREG * mid2) / (2 * total) : 0;
  return int32_t(r < 0 ? 0 : (r >= NREG ? NREG - 1 : r));
}

// smallest and largest key of every region (bounds[2r], bounds[2r+1]; an
// empty region keeps the pair k_bounds_init wrote).  region_of never
// decreases with k (the prefix sums only grow), so a region's keys are one
// range and its ends are the keys where the region changes.
__global__ void k_region_bounds(const int32_t* pre, const int32_t* w, int32_t nkeys, int64_t total,
                                int32_t* bounds) {
  const int32_t k = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int32_t r = region_of(pre, w, k, total);
  if (k == 0 || region_of(pre, w, k - 1, total) != r) bounds[2 * r] = k;
  if (k == nkeys - 1 || region_of(pre, w, k + 1, total) != r) bounds[2 * r + 1] = k;
}

// entries per batch of loads in the one-thread-per-row kernels below (indices
// clamped to the row: no branch, all loads of a batch in flight together)
constexpr int ROW_BATCH = 8;

// key of every row: the smallest key of its entries; short rows one thread
// each, projection rows one wave each
__global__ void k_row_keys(const int32_t* rrow_ptr, const uint32_t* word, const int32_t* vkey, int64_t n_rows,
                           int32_t* rkey) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_rows) return;
  int32_t m = INT32_MAX;
  const int32_t s = rrow_ptr[j], t = rrow_ptr[j + 1];
  for (int32_t e0 = s; e0 < t; e0 += ROW_BATCH) {   // the loads of a batch go out together
    uint32_t w[ROW_BATCH];
#pragma unroll
    for (int u = 0; u < ROW_BATCH; ++u) w[u] = word[e0 + u < t ? e0 + u : e0];
#pragma unroll
    for (int u = 0; u < ROW_BATCH; ++u) m = min(m, vkey[w[u] & W_VAR_MASK]);   // repeats of e0 change nothing
  }
  rkey[j] = m == INT32_MAX ? 0 : m;
}

__global__ void k_long_row_keys(const int32_t* rrow_ptr, const uint32_t* word, const int32_t* vkey, int64_t n_short,
                                int64_t n_rows, int32_t* rkey) {
  const int64_t j = n_short + int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n_rows) return;   // uniform across the wave
  const int lane = threadIdx.x & 63;
  int32_t m = INT32_MAX;
  for (int32_t e = rrow_ptr[j] + lane; e < rrow_ptr[j + 1]; e += 64) m = min(m, vkey[word[e] & W_VAR_MASK]);
  for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off));
  if (lane == 0) rkey[j] = m == INT32_MAX ? 0 : m;
}

// short rows: sort key (tile row or not, row key), sorted stably so that
// equal keys keep the row order.  Rows with b = 0 and at most TILE_HALF
// entries of each sign go first (they run one lane per row in 64-row tiles),
// the others follow; both in key order.  Bit kbits marks the others.
constexpr int TILE_HALF = 8;
constexpr int TILE_WORDS = 2 * TILE_HALF * 64;
// Tiles cut the sweep's vector instructions several times over, but a tile
// wave touches the records of 64 rows at once: on problems of more than
// TILE_NNZ_MAX nonzeros (records well past what the L2s and the Infinity
// Cache hold) the wider footprint costs more in record traffic than the
// instructions save, and all short rows stay in chunks (2000/3000-face pair,
// 17.8 M nonzeros: 250 us with tiles, 260 us in chunks; the same geometry
// with 52.7 M nonzeros: 875 us with tiles, 839 us in chunks).
constexpr int64_t TILE_NNZ_MAX = int64_t(24) << 20;

__global__ void k_short_sort_keys(const int32_t* rkey, const int32_t* rrow_ptr, const int32_t* rrow_b,
                                  const uint32_t* word, int64_t n_short, int tiles_on, int kbits, uint32_t* key,
                                  int32_t* val,
                                  int32_t* n_tile_rows /* [2]: rows, entries */) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_short) return;
  const int32_t s = rrow_ptr[j], t = rrow_ptr[j + 1];
  int32_t nq = 0;
  for (int32_t e0 = s; e0 < t; e0 += ROW_BATCH) {   // the loads of a batch go out together
    uint32_t w[ROW_BATCH];
#pragma unroll
    for (int u = 0; u < ROW_BATCH; ++u) w[u] = word[e0 + u < t ? e0 + u : e0];
#pragma unroll
    for (int u = 0; u < ROW_BATCH; ++u) nq += (e0 + u < t && (w[u] & W_NEG)) ? 1 : 0;
  }
  const int32_t np = (t - s) - nq;
  const bool tile = tiles_on && rrow_b[j] == 0 && np <= TILE_HALF && nq <= TILE_HALF;
  key[j] = (tile ? 0u : (1u << kbits)) | uint32_t(rkey[j]);
  val[j] = int32_t(j);
  if (tile) {
    atomicAdd(&n_tile_rows[0], 1);
    atomicAdd(&n_tile_rows[1], np + nq);   // their entries
  }
}

// words of every tile row into its lane of its tile: +1 entries in slots 0 to
// TILE_HALF - 1, -1 entries in the next TILE_HALF slots, each in row order
__global__ void k_tile_fill(const int32_t* perm, int64_t n_tile_rows, const int32_t* rrow_ptr,
                            const uint32_t* word, uint32_t* tile_word) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_tile_rows) return;
  uint32_t* dst = tile_word + size_t(k / 64) * TILE_WORDS + size_t(k % 64);
  const int32_t j = perm[k];
  int32_t np = 0, nq = 0;
  for (int32_t e = rrow_ptr[j]; e < rrow_ptr[j + 1]; ++e) {
    const uint32_t w = word[e];
    if (w & W_NEG) dst[size_t(TILE_HALF + nq++) * 64] = w;
    else dst[size_t(np++) * 64] = w;
  }
}

// long rows: sort key (region, key), sorted stably (equal keys keep the row
// order); an X projection row (or any long row of a generic problem) takes
// its own key's region; the o-th Y projection row goes to region o % 8 at a
// key spread over that region's range.  Long rows whose full row index
// (rrow_orig) is at least first_y_full are Y projection rows; *first_y_long
// counts the long rows before them.
__global__ void k_count_below(const int32_t* rrow_orig, int64_t n_short, int64_t n_long, int64_t first_y_full,
                              int32_t* count) {
  const int64_t l = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (l < n_long && rrow_orig[n_short + l] < first_y_full) atomicAdd(count, 1);
}

__global__ void k_long_sort_keys(const int32_t* rkey, const int32_t* rrow_orig, int64_t n_short, int64_t n_long,
                                 int64_t first_y_full, const int32_t* first_y_long, int kbits, const int32_t* pre,
                                 const int32_t* w, int64_t total, const int32_t* bounds, uint32_t* key,
                                 int32_t* val) {
  const int64_t l = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (l >= n_long) return;
  const int64_t j = n_short + l;
  int32_t r, k;
  if (rrow_orig[j] < first_y_full) {
    k = rkey[j];
    r = region_of(pre, w, k, total);
  } else {
    const int64_t fy = *first_y_long, n_y = n_long - fy;
    const int64_t o = l - fy;
    r = int32_t(o % NREG);
    const int64_t per = (n_y - r + NREG - 1) / NREG;   // Y rows of region r
    const int32_t lo = bounds[2 * r], hi = bounds[2 * r + 1];
    const int64_t span = hi >= lo ? int64_t(hi) - lo + 1 : 1;
    k = int32_t((hi >= lo ? lo : 0) + ((o / NREG) * span) / (per > 0 ? per : 1));
  }
  key[l] = (uint32_t(r) << kbits) | uint32_t(k);
  val[l] = int32_t(l);
}

// ---------------------------------------------------------------- short rows in key order
__global__ void k_perm_len(const int32_t* perm, const int32_t* rrow_ptr, const int32_t* rrow_b, int64_t n,
                           int32_t* len, int32_t* pb) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t j = perm[k];
  len[k] = rrow_ptr[j + 1] - rrow_ptr[j];
  pb[k] = rrow_b[j];
}

__global__ void k_gather_i32(const int32_t* perm, const int32_t* src, int64_t n, int32_t* dst) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[perm[k]];
}

__global__ void k_perm_words(const int32_t* perm, const int32_t* rrow_ptr, const int32_t* prow_ptr,
                             const uint32_t* word, int64_t n, uint32_t* pword) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t j = perm[k], s = rrow_ptr[j], o = prow_ptr[k], m = rrow_ptr[j + 1] - s;
  for (int32_t e = 0; e < m; ++e) pword[o + e] = word[s + e];
}

// Rows are packed greedily, in order, into wave chunks of at most 64 entries
// (one entry per lane, whole rows only).  The greedy walk runs in parallel
// over segments of PACK_SEG entries: segment j holds the rows whose first
// entry lies in [j*PACK_SEG, (j+1)*PACK_SEG).
__global__ void k_seg_rows(const int32_t* row_ptr, int64_t n_rows, int32_t n_seg, int32_t* seg_row) {
  int32_t j = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j > n_seg) return;
  if (j == n_seg) {
    seg_row[j] = int32_t(n_rows);
    return;
  }
  int64_t target = int64_t(j) * PACK_SEG;
  int64_t lo = 0, hi = n_rows;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (row_ptr[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  seg_row[j] = int32_t(lo);
}

// One block per segment: the segment's row pointers are staged in LDS (a
// segment starts at most PACK_SEG / 2 rows, since every presolved row has at
// least two entries), then one thread walks them.  fill == 0: count the
// chunks of each segment; fill == 1: write their (first row, rows, first
// entry, entries) at the scanned offsets.
__global__ __launch_bounds__(256) void k_pack(const int32_t* seg_row, const int32_t* row_ptr, int32_t n_seg,
                                              int32_t* count, const int32_t* offset, int4* desc, int fill) {
  __shared__ int32_t rp[PACK_SEG / 2 + 1];
  const int32_t j = blockIdx.x;
  const int32_t rs = seg_row[j], nr = seg_row[j + 1] - rs;
  if (nr > PACK_SEG / 2) return;   // excluded by the caller's check
  for (int32_t i = threadIdx.x; i <= nr; i += blockDim.x) rp[i] = row_ptr[rs + i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t r = 0, c = 0, o = fill ? offset[j] : 0;
  while (r < nr) {
    const int32_t q0 = r, e0 = rp[r];
    // extend the chunk while the next row still fits, eight row pointers per step
    for (;;) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = r + 1 + u <= nr ? rp[r + 1 + u] : INT32_MAX;
      int adv = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (adv == u && r + u < nr && v[u] - e0 <= 64) adv = u + 1;
      r += adv;
      if (adv < 8) break;
    }
    if (fill) desc[o + c] = make_int4(rs + q0, r - q0, e0, rp[r] - e0);
    ++c;
  }
  if (!fill) count[j] = c;
}

// per chunk, the positions (relative to its first entry) where its rows start
__global__ void k_chunk_mask(const int4* desc, const int32_t* row_ptr, int32_t n_chunks,
                             unsigned long long* mask) {
  const int32_t c = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= n_chunks) return;
  const int4 d = desc[c];
  unsigned long long m = 0ull;
  for (int32_t r = 0; r < d.y; ++r) m |= 1ull << (row_ptr[d.x + r] - d.z);
  mask[c] = m;
}

// padded copy of every chunk: 64 entry words (CHUNK_PAD past the chunk's end)
// and the right-hand side of each entry's row, so that a wave reads its
// entries without first reading the chunk descriptor
__global__ void k_chunk_pad(const int4* desc, const unsigned long long* mask, const uint32_t* word,
                            const int32_t* row_b, int32_t n_chunks, uint32_t* pword, int8_t* pb) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n_chunks) * 64) return;
  const int32_t c = int32_t(t >> 6), e = int32_t(t & 63);
  const int4 d = desc[c];
  if (e < d.w) {
    const unsigned long long below = mask[c] & (e == 63 ? ~0ull : ((2ull << e) - 1ull));
    pword[t] = word[d.z + e];
    pb[t] = int8_t(row_b[d.x + __popcll(below) - 1]);
  } else {
    pword[t] = CHUNK_PAD;
    pb[t] = 0;
  }
}

// ---------------------------------------------------------------- items and the per-XCD table
// item keys: a tile item (four tiles) takes the region and key of its first
// row, a chunk item (four chunks) those of its first row, a long item those
// of its first long row.  Items are numbered [tile items | chunk items | long
// items].
__global__ void k_item_keys(int32_t n_tile_items, const uint32_t* skey, uint32_t kmask, const int4* desc,
                            int32_t n_chunk_items, const int32_t* prkey, const int32_t* pre, const int32_t* w,
                            int64_t total, const uint32_t* lkey_sorted, int32_t n_long_items, int32_t rows_per_long,
                            int kbits, uint32_t* key, int32_t* val) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_tile_items + n_chunk_items + n_long_items) return;
  uint32_t r, k;
  if (i < n_tile_items) {
    k = skey[int64_t(i) * 256] & kmask;
    r = uint32_t(region_of(pre, w, int32_t(k), total));
  } else if (i < n_tile_items + n_chunk_items) {
    k = uint32_t(prkey[desc[4 * (i - n_tile_items)].x]);
    r = uint32_t(region_of(pre, w, int32_t(k), total));
  } else {
    const uint32_t lk = lkey_sorted[int64_t(i - n_tile_items - n_chunk_items) * rows_per_long];
    r = lk >> kbits;
    k = lk & kmask;
  }
  key[i] = (r << kbits) | k;
  val[i] = i;
}

__global__ void k_region_count(const uint32_t* key, int32_t n, int kbits, int32_t* cnt) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[int(key[i] >> kbits)], 1);
}

__global__ void k_xcd_table(const int32_t* sorted_item, int32_t n_items, const int32_t* start, int32_t stride,
                            int32_t* table) {
  const int32_t t = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= NREG * stride) return;
  const int32_t x = t / stride, k = t % stride;
  const int32_t a = start[x] + k;
  table[t] = a < start[x + 1] ? sorted_item[a] : -1;
}

}  // namespace

// mean projection-row length above which a projection row gets a whole block
constexpr int64_t LONG_BLOCK_ROW = 512;

dm_status sweep_layout(dm_ctx* ctx) {
  hipStream_t st = ctx->stream;
  const int64_t nfree = ctx->n_free, nr = ctx->n_rows, nshort = ctx->n_short, rnnz = ctx->nnz;
  const int64_t nlong = nr - nshort;
  // ---- variable keys
  const bool mesh = !ctx->generic && ctx->X.nf > 0;
  const int32_t nkeys = mesh ? ctx->X.nf : int32_t(std::max<int64_t>(nfree, 1));
  DArr<int32_t> vkey, wcount, wpre, bounds, rkey;
  DM_ALLOC(ctx, vkey, size_t(std::max<int64_t>(nfree, 1)));
  if (mesh) {
    MeshDev& X = ctx->X;
    DArr<float> box;
    DArr<uint32_t> fkey;
    DArr<int32_t> forder, frank, erank, vrank;
    DM_ALLOC(ctx, box, 6);
    DM_ALLOC(ctx, fkey, size_t(X.nf));
    DM_ALLOC(ctx, forder, size_t(X.nf));
    DM_ALLOC(ctx, frank, size_t(X.nf));
    DM_ALLOC(ctx, erank, size_t(X.ne));
    DM_ALLOC(ctx, vrank, size_t(X.nv));
    k_bbox<<<1, 256, 0, st>>>(X.verts.p, X.nv, box.p);
    k_face_morton<<<grid_for(X.nf, 256), 256, 0, st>>>(X.verts.p, X.faces.p, X.nf, box.p, fkey.p, forder.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, fkey.p, forder.p, size_t(X.nf), 30));
    k_rank_of<<<grid_for(X.nf, 256), 256, 0, st>>>(forder.p, X.nf, frank.p);
    k_fill_i32<<<grid_for(X.ne, 256), 256, 0, st>>>(erank.p, X.ne, INT32_MAX);
    k_fill_i32<<<grid_for(X.nv, 256), 256, 0, st>>>(vrank.p, X.nv, INT32_MAX);
    k_elem_rank<<<grid_for(X.nf, 256), 256, 0, st>>>(X.faces.p, X.face_edge.p, frank.p, X.nf, erank.p, vrank.p);
    if (nfree > 0)
      k_var_key_mesh<<<grid_for(nfree, 256), 256, 0, st>>>(ctx->free_var.p, ctx->code.p, frank.p, erank.p,
                                                           vrank.p, nfree, vkey.p);
    DM_LAUNCH_CHECK(ctx);
  } else if (nfree > 0) {
    k_iota<<<grid_for(nfree, 256), 256, 0, st>>>(vkey.p, nfree);
    DM_LAUNCH_CHECK(ctx);
  }
  // ---- regions: eight key ranges of equal entry counts
  DM_ALLOC(ctx, wcount, size_t(nkeys));
  DM_ALLOC(ctx, wpre, size_t(nkeys) + 1);
  DM_ALLOC(ctx, bounds, 2 * NREG);
  DM_HIP(ctx, hipMemsetAsync(wcount.p, 0, sizeof(int32_t) * nkeys, st));
  if (mesh && nfree > 0) {
    if (nkeys > KEY_BINS_LDS)
      return dm_fail(ctx, DM_ERR_WORKSPACE, "sweep layout: %d faces exceed %d key bins", nkeys, KEY_BINS_LDS);
    k_key_weight<<<grid_for(nfree, KEY_VARS_PER_BLOCK), 256, size_t(nkeys) * sizeof(int32_t), st>>>(
        vkey.p, ctx->var_deg.p, nfree, nkeys, wcount.p);
  } else if (nfree > 0) {
    k_deg_weight<<<grid_for(nfree, 256), 256, 0, st>>>(ctx->var_deg.p, nfree, wcount.p);
  }
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_i32(ctx, wcount.p, wpre.p, size_t(nkeys)));
  k_bounds_init<<<1, 64, 0, st>>>(bounds.p);
  k_region_bounds<<<grid_for(nkeys, 256), 256, 0, st>>>(wpre.p, wcount.p, nkeys, rnnz, bounds.p);
  DM_ALLOC(ctx, rkey, size_t(std::max<int64_t>(nr, 1)));
  if (nshort > 0)
    k_row_keys<<<grid_for(nshort, 256), 256, 0, st>>>(ctx->rrow_ptr.p, ctx->rent_word.p, vkey.p, nshort, rkey.p);
  if (nlong > 0)
    k_long_row_keys<<<grid_for(nlong, 4), 256, 0, st>>>(ctx->rrow_ptr.p, ctx->rent_word.p, vkey.p, nshort, nr,
                                                         rkey.p);
  DM_LAUNCH_CHECK(ctx);

  // ---- short rows: 64-row tiles of b = 0 rows, then the rest in wave chunks, both in key order
  // stable radix sorts on compact keys: keys take kbits bits, one more bit
  // marks non-tile rows, three more bits above them hold the region
  const int kbits = bits_for(uint64_t(nkeys));
  const uint32_t kmask = (1u << kbits) - 1u;
  DArr<uint32_t> skey;
  DArr<int32_t> perm, plen, prow_ptr, pb, prkey, ntr;
  DArr<uint32_t> pword;
  DM_ALLOC(ctx, skey, size_t(std::max<int64_t>(nshort, 1)));
  DM_ALLOC(ctx, perm, size_t(std::max<int64_t>(nshort, 1)));
  DM_ALLOC(ctx, ntr, 2);
  DM_HIP(ctx, hipMemsetAsync(ntr.p, 0, 2 * sizeof(int32_t), st));
  if (nshort > 0) {
    k_short_sort_keys<<<grid_for(nshort, 256), 256, 0, st>>>(rkey.p, ctx->rrow_ptr.p, ctx->rrow_b.p,
                                                             ctx->rent_word.p, nshort, rnnz <= TILE_NNZ_MAX ? 1 : 0,
                                                             kbits, skey.p, perm.p, ntr.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, skey.p, perm.p, size_t(nshort), kbits + 1));
  }
  int32_t n_tile_rows = 0, nnz_chunk = 0;
  {
    const int32_t* src[2] = {ntr.p, ntr.p + 1};
    int32_t v[2];
    DM_TRY(read_i32s(ctx, 2, src, v));
    n_tile_rows = v[0];
    nnz_chunk = int32_t(ctx->nnz_short) - v[1];   // entries of the short rows left to the chunks
  }
  ctx->n_tiles = (n_tile_rows + 63) / 64;
  ctx->n_tile_items = (ctx->n_tiles + 3) / 4;
  const size_t twords = size_t(ctx->n_tiles) * TILE_WORDS;
  DM_ALLOC(ctx, ctx->tile_word, std::max<size_t>(twords, 1));
  DM_HIP(ctx, hipMemsetAsync(ctx->tile_word.p, 0xFF, sizeof(uint32_t) * std::max<size_t>(twords, 1), st));
  if (n_tile_rows > 0)
    k_tile_fill<<<grid_for(n_tile_rows, 256), 256, 0, st>>>(perm.p, n_tile_rows, ctx->rrow_ptr.p,
                                                            ctx->rent_word.p, ctx->tile_word.p);
  DM_LAUNCH_CHECK(ctx);
  // the remaining short rows in key order, packed into wave chunks
  const int64_t nchr = nshort - n_tile_rows;
  const int32_t* cperm = perm.p + n_tile_rows;
  DM_ALLOC(ctx, plen, size_t(std::max<int64_t>(nchr, 1)));
  DM_ALLOC(ctx, pb, size_t(std::max<int64_t>(nchr, 1)));
  DM_ALLOC(ctx, prkey, size_t(std::max<int64_t>(nchr, 1)));
  DM_ALLOC(ctx, prow_ptr, size_t(nchr) + 1);
  if (nchr > 0) {
    k_perm_len<<<grid_for(nchr, 256), 256, 0, st>>>(cperm, ctx->rrow_ptr.p, ctx->rrow_b.p, nchr, plen.p, pb.p);
    k_gather_i32<<<grid_for(nchr, 256), 256, 0, st>>>(cperm, rkey.p, nchr, prkey.p);
    DM_LAUNCH_CHECK(ctx);
  }
  DM_TRY(scan_i32(ctx, plen.p, prow_ptr.p, size_t(nchr)));
  DM_ALLOC(ctx, pword, size_t(std::max(nnz_chunk, 1)));
  if (nchr > 0) {
    k_perm_words<<<grid_for(nchr, 256), 256, 0, st>>>(cperm, ctx->rrow_ptr.p, prow_ptr.p, ctx->rent_word.p, nchr,
                                                      pword.p);
    DM_LAUNCH_CHECK(ctx);
  }
  const int32_t n_seg = int32_t((int64_t(nnz_chunk) + PACK_SEG - 1) / PACK_SEG);
  DArr<int32_t> seg_row, seg_cnt, seg_off;
  DM_ALLOC(ctx, seg_row, size_t(n_seg) + 1);
  DM_ALLOC(ctx, seg_cnt, size_t(std::max(n_seg, 1)));
  DM_ALLOC(ctx, seg_off, size_t(n_seg) + 1);
  k_seg_rows<<<grid_for(n_seg + 1, 256), 256, 0, st>>>(prow_ptr.p, nchr, n_seg, seg_row.p);
  if (n_seg > 0)
    k_pack<<<unsigned(n_seg), 256, 0, st>>>(seg_row.p, prow_ptr.p, n_seg, seg_cnt.p, nullptr, nullptr, 0);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_i32(ctx, seg_cnt.p, seg_off.p, size_t(n_seg)));
  int32_t n_chunks = 0;
  DM_TRY(read_i32(ctx, seg_off.p + n_seg, &n_chunks));
  ctx->n_chunks = n_chunks;
  DM_ALLOC(ctx, ctx->chunk_desc, size_t(std::max(n_chunks, 1)));
  if (n_seg > 0)
    k_pack<<<unsigned(n_seg), 256, 0, st>>>(seg_row.p, prow_ptr.p, n_seg, nullptr, seg_off.p, ctx->chunk_desc.p,
                                            1);
  DM_ALLOC(ctx, ctx->chunk_mask, size_t(std::max(n_chunks, 1)));
  if (n_chunks > 0)
    k_chunk_mask<<<grid_for(n_chunks, 256), 256, 0, st>>>(ctx->chunk_desc.p, prow_ptr.p, n_chunks,
                                                          ctx->chunk_mask.p);
  DM_ALLOC(ctx, ctx->chunk_word, size_t(std::max(n_chunks, 1)) * 64);
  DM_ALLOC(ctx, ctx->chunk_b, size_t(std::max(n_chunks, 1)) * 64);
  if (n_chunks > 0)
    k_chunk_pad<<<grid_for(int64_t(n_chunks) * 64, 256), 256, 0, st>>>(
        ctx->chunk_desc.p, ctx->chunk_mask.p, pword.p, pb.p, n_chunks, ctx->chunk_word.p, ctx->chunk_b.p);
  DM_LAUNCH_CHECK(ctx);

  // ---- projection rows: one wave each, or a whole block each when they are long
  ctx->long_wpr = (nlong > 0 && (rnnz - ctx->nnz_short) / nlong > LONG_BLOCK_ROW) ? 4 : 1;
  const int32_t rows_per_long = 4 / ctx->long_wpr;
  const int32_t n_long_items = int32_t((nlong + rows_per_long - 1) / rows_per_long);
  const int32_t n_chunk_items = (n_chunks + 3) / 4;
  DArr<uint32_t> lkey;
  DArr<int32_t> fyl;
  DM_ALLOC(ctx, lkey, size_t(std::max<int64_t>(nlong, 1)));
  DM_ALLOC(ctx, fyl, 1);
  DM_ALLOC(ctx, ctx->long_perm, size_t(std::max<int64_t>(nlong, 1)));
  if (nlong > 0) {
    // Y projection rows follow the X ones: count the long rows of a full
    // index below the first Y projection row
    const int64_t first_y_full = mesh ? ctx->n_closed_full + ctx->X.nf : INT64_MAX;
    DM_HIP(ctx, hipMemsetAsync(fyl.p, 0, sizeof(int32_t), st));
    k_count_below<<<grid_for(nlong, 256), 256, 0, st>>>(ctx->rrow_orig.p, nshort, nlong, first_y_full, fyl.p);
    k_long_sort_keys<<<grid_for(nlong, 256), 256, 0, st>>>(rkey.p, ctx->rrow_orig.p, nshort, nlong, first_y_full,
                                                           fyl.p, kbits, wpre.p, wcount.p, rnnz, bounds.p, lkey.p,
                                                           ctx->long_perm.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, lkey.p, ctx->long_perm.p, size_t(nlong), kbits + 3));
  }

  // ---- items in (region, key) order and the per-XCD table
  const int32_t n_items = ctx->n_tile_items + n_chunk_items + n_long_items;
  ctx->n_long_items = n_long_items;
  DArr<uint32_t> ikey;
  DArr<int32_t> iorder, cnt;
  DM_ALLOC(ctx, ikey, size_t(std::max(n_items, 1)));
  DM_ALLOC(ctx, iorder, size_t(std::max(n_items, 1)));
  DM_ALLOC(ctx, cnt, NREG);
  DM_HIP(ctx, hipMemsetAsync(cnt.p, 0, NREG * sizeof(int32_t), st));
  if (n_items > 0) {
    k_item_keys<<<grid_for(n_items, 256), 256, 0, st>>>(ctx->n_tile_items, skey.p, kmask, ctx->chunk_desc.p,
                                                        n_chunk_items, prkey.p, wpre.p, wcount.p, rnnz, lkey.p,
                                                        n_long_items, rows_per_long, kbits, ikey.p, iorder.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, ikey.p, iorder.p, size_t(n_items), kbits + 3));
    k_region_count<<<grid_for(n_items, 256), 256, 0, st>>>(ikey.p, n_items, kbits, cnt.p);
    DM_LAUNCH_CHECK(ctx);
  }
  int32_t hc[NREG];
  DM_HIP(ctx, hipMemcpyAsync(hc, cnt.p, sizeof(hc), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  int32_t start[NREG + 1], stride = 0;
  start[0] = 0;
  for (int r = 0; r < NREG; ++r) {
    start[r + 1] = start[r] + hc[r];
    stride = std::max(stride, hc[r]);
  }
  ctx->xcd_stride = stride;
  DArr<int32_t> dstart;
  DM_ALLOC(ctx, dstart, NREG + 1);
  DM_HIP(ctx, hipMemcpyAsync(dstart.p, start, sizeof(start), hipMemcpyHostToDevice, st));
  DM_ALLOC(ctx, ctx->xcd_item, size_t(std::max(NREG * stride, 1)));
  if (stride > 0)
    k_xcd_table<<<grid_for(NREG * stride, 256), 256, 0, st>>>(iorder.p, n_items, dstart.p, stride,
                                                              ctx->xcd_item.p);
  DM_LAUNCH_CHECK(ctx);
  // the host copy of start[] must outlive the copy above
  DM_HIP(ctx, hipStreamSynchronize(st));
  return DM_OK;
}
