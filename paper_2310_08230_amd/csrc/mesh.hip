// Mesh ingest (validation, edge table) and mixed vertex areas.
//
// A mesh (Table "notation") must be a closed, oriented 2-manifold: every
// directed edge occurs once and its reverse once, and the faces around each
// vertex form a single fan.  Edges are numbered by their sorted (min, max)
// vertex pairs.  Only closed meshes of equal genus admit a solution of (P)
// (Sec. 5 "Datasets").
#include <cmath>

#include "dm_internal.h"

enum : int { ERR_RANGE = 1, ERR_DEGEN = 2, ERR_DUP = 4, ERR_OPEN = 8, ERR_UNUSED = 16,
             ERR_FAN = 32, ERR_NONFINITE = 64 };

__device__ inline int64_t lower_bound_u64(const uint64_t* a, int64_t n, uint64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_check_finite(const float* v, int64_t n, int* err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) atomicOr(err, ERR_NONFINITE);
}

__global__ void k_dirkeys(const int32_t* F, int32_t nf, int32_t nv, uint64_t* key, int32_t* val,
                          int* err) {
  int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= int64_t(nf) * 3) return;
  int64_t f = c / 3;
  int k = int(c % 3);
  int32_t a = F[3 * f + k], b = F[3 * f + (k + 1) % 3], o = F[3 * f + (k + 2) % 3];
  bool ok = a >= 0 && a < nv && b >= 0 && b < nv && o >= 0 && o < nv;
  if (!ok) atomicOr(err, ERR_RANGE);
  else if (a == b || b == o || a == o) atomicOr(err, ERR_DEGEN);
  key[c] = ok ? uint64_t(a) * uint64_t(nv) + uint64_t(b) : ~uint64_t(0);
  val[c] = int32_t(c);
}

__global__ void k_edge_check(const uint64_t* key, int64_t n, int32_t nv, uint8_t* lower, int* err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = key[i];
  if (k == ~uint64_t(0)) {
    lower[i] = 0;
    return;
  }
  if (i > 0 && key[i - 1] == k) atomicOr(err, ERR_DUP);
  uint64_t a = k / uint64_t(nv), b = k % uint64_t(nv);
  uint64_t r = b * uint64_t(nv) + a;
  int64_t pos = lower_bound_u64(key, n, r);
  if (pos >= n || key[pos] != r) atomicOr(err, ERR_OPEN);
  lower[i] = a < b ? 1 : 0;
}

__global__ void k_edges(const uint64_t* key, const int32_t* val, int64_t n, int32_t nv,
                        const int32_t* eid, int32_t* edges, int32_t* face_edge) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = key[i];
  uint64_t a = k / uint64_t(nv), b = k % uint64_t(nv);
  int32_t id;
  if (a < b) {
    id = eid[i];
    edges[2 * id] = int32_t(a);
    edges[2 * id + 1] = int32_t(b);
  } else {
    int64_t pos = lower_bound_u64(key, n, b * uint64_t(nv) + a);
    id = eid[pos];
  }
  face_edge[val[i]] = id;
}

__global__ void k_vertex_fan(const uint64_t* key, const int32_t* val, int64_t n, const int32_t* F,
                             int32_t nv, int* err) {
  int32_t v = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int64_t s = lower_bound_u64(key, n, uint64_t(v) * uint64_t(nv));
  int64_t e = lower_bound_u64(key, n, uint64_t(v + 1) * uint64_t(nv));
  int64_t deg = e - s;
  if (deg <= 0) {
    atomicOr(err, ERR_UNUSED);
    return;
  }
  int64_t pos = s, count = 0;
  do {
    int32_t c = val[pos];
    int32_t f = c / 3, k = c % 3;
    int32_t u = F[3 * f + (k + 2) % 3];          // u -> v lies in f; v -> u starts the next face
    uint64_t nk = uint64_t(v) * uint64_t(nv) + uint64_t(u);
    pos = lower_bound_u64(key, n, nk);
    ++count;
    if (pos >= n || key[pos] != nk || count > deg) {
      atomicOr(err, ERR_FAN);
      return;
    }
  } while (pos != s);
  if (count != deg) atomicOr(err, ERR_FAN);
}

static dm_status mesh_error(dm_ctx* ctx, int e, const char* name) {
  if (e & ERR_NONFINITE) return dm_fail(ctx, DM_ERR_NONFINITE, "mesh %s: non-finite vertex", name);
  if (e & ERR_RANGE) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: face index out of range", name);
  if (e & ERR_DEGEN) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: face repeats a vertex", name);
  if (e & ERR_DUP) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: directed edge used twice", name);
  if (e & ERR_OPEN) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: open or inconsistently oriented edge", name);
  if (e & ERR_UNUSED) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: unused vertex", name);
  if (e & ERR_FAN) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: vertex is not manifold", name);
  return DM_OK;
}

dm_status mesh_ingest(dm_ctx* ctx, const dm_mesh* in, MeshDev& m, const char* name) {
  if (!in || !in->verts || !in->faces)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "mesh %s: NULL pointer", name);
  if (in->nv < 3 || in->nf < 1 || in->nv > 46340)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "mesh %s: nv=%d nf=%d outside [3, 46340] x [1, ...)",
                   name, in->nv, in->nf);
  const int32_t nv = in->nv, nf = in->nf;
  const int64_t nc = int64_t(nf) * 3;
  m.nv = nv;
  m.nf = nf;
  DM_ALLOC(ctx, m.verts, size_t(nv) * 3);
  DM_ALLOC(ctx, m.faces, size_t(nc));
  DM_HIP(ctx, hipMemcpyAsync(m.verts.p, in->verts, sizeof(float) * 3 * nv, hipMemcpyDeviceToDevice,
                             ctx->stream));
  DM_HIP(ctx, hipMemcpyAsync(m.faces.p, in->faces, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice,
                             ctx->stream));
  DArr<int> err;
  DM_ALLOC(ctx, err, 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), ctx->stream));
  k_check_finite<<<grid_for(int64_t(nv) * 3, 256), 256, 0, ctx->stream>>>(m.verts.p, int64_t(nv) * 3, err.p);
  DM_ALLOC(ctx, m.dkey, size_t(nc));
  DM_ALLOC(ctx, m.dval, size_t(nc));
  k_dirkeys<<<grid_for(nc, 256), 256, 0, ctx->stream>>>(m.faces.p, nf, nv, m.dkey.p, m.dval.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  // no read back yet: a face with an index out of range gets the all-ones
  // key, which the sort, the edge check and the scan handle within bounds,
  // and the errors flagged so far are read with the edge count below (the
  // report takes the first error in a fixed order, so it names the same one)
  int e = 0;
  DM_TRY(sort_pairs_u64(ctx, m.dkey.p, m.dval.p, size_t(nc), bits_for(uint64_t(nv) * nv)));
  DArr<uint8_t> lower;
  DArr<int32_t> eid;
  DM_ALLOC(ctx, lower, size_t(nc));
  DM_ALLOC(ctx, eid, size_t(nc) + 1);
  k_edge_check<<<grid_for(nc, 256), 256, 0, ctx->stream>>>(m.dkey.p, nc, nv, lower.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, lower.p, eid.p, size_t(nc)));
  int32_t ne = 0;
  {
    const int32_t* src[2] = {err.p, eid.p + nc};
    int32_t v[2];
    DM_TRY(read_i32s(ctx, 2, src, v));
    e = v[0];
    ne = v[1];
  }
  if (e) return mesh_error(ctx, e, name);
  m.ne = ne;
  if (int64_t(ne) * 2 != nc) return dm_fail(ctx, DM_ERR_MESH, "mesh %s: not closed", name);
  DM_ALLOC(ctx, m.edges, size_t(ne) * 2);
  DM_ALLOC(ctx, m.face_edge, size_t(nc));
  k_edges<<<grid_for(nc, 256), 256, 0, ctx->stream>>>(m.dkey.p, m.dval.p, nc, nv, eid.p, m.edges.p,
                                                      m.face_edge.p);
  k_vertex_fan<<<grid_for(nv, 256), 256, 0, ctx->stream>>>(m.dkey.p, m.dval.p, nc, m.faces.p, nv, err.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(read_i32(ctx, err.p, &e));
  if (e) return mesh_error(ctx, e, name);
  return DM_OK;
}

// ---------------------------------------------------------------------------
// Mixed (Voronoi) areas, Meyer et al. 2003 (the area weights of Eq. (cost),
// Sec. 4.2).  Per corner p of triangle (p, q, r): in a triangle with no obtuse
// angle, (|pq|^2 cot(angle r) + |pr|^2 cot(angle q)) / 8; in an obtuse triangle,
// half its area at the obtuse corner and a quarter at the other two.  The
// per-vertex sum runs over the vertex's corners in sorted outgoing-edge order.
// ---------------------------------------------------------------------------
__global__ void k_corner_area(const float* V, const int32_t* F, int32_t nf, double* contrib) {
  int32_t f = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) P[k][c] = double(V[3 * int64_t(F[3 * f + k]) + c]);
  double e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = P[1][c] - P[0][c];
    e2[c] = P[2][c] - P[0][c];
  }
  double cx = e1[1] * e2[2] - e1[2] * e2[1];
  double cy = e1[2] * e2[0] - e1[0] * e2[2];
  double cz = e1[0] * e2[1] - e1[1] * e2[0];
  double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
  double dotk[3];
  for (int k = 0; k < 3; ++k) {
    const double* p = P[k];
    const double* q = P[(k + 1) % 3];
    const double* r = P[(k + 2) % 3];
    dotk[k] = (q[0] - p[0]) * (r[0] - p[0]) + (q[1] - p[1]) * (r[1] - p[1]) + (q[2] - p[2]) * (r[2] - p[2]);
  }
  bool obtuse = dotk[0] < 0.0 || dotk[1] < 0.0 || dotk[2] < 0.0;
  for (int k = 0; k < 3; ++k) {
    double a;
    if (!obtuse) {
      int q = (k + 1) % 3, r = (k + 2) % 3;
      // cot(angle at r) = dot / (2 area) of the edges leaving r, same at q
      double cot_r = dotk[r] / (2.0 * area);
      double cot_q = dotk[q] / (2.0 * area);
      double lpq = 0.0, lpr = 0.0;
      for (int c = 0; c < 3; ++c) {
        lpq += (P[q][c] - P[k][c]) * (P[q][c] - P[k][c]);
        lpr += (P[r][c] - P[k][c]) * (P[r][c] - P[k][c]);
      }
      a = (lpq * cot_r + lpr * cot_q) / 8.0;
    } else {
      a = dotk[k] < 0.0 ? area / 2.0 : area / 4.0;
    }
    contrib[3 * int64_t(f) + k] = a;
  }
}

__global__ void k_vertex_area(const uint64_t* key, const int32_t* val, int64_t n, int32_t nv,
                              const double* contrib, double* area) {
  int32_t v = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int64_t s = lower_bound_u64(key, n, uint64_t(v) * uint64_t(nv));
  int64_t e = lower_bound_u64(key, n, uint64_t(v + 1) * uint64_t(nv));
  double a = 0.0;
  for (int64_t i = s; i < e; ++i) a += contrib[val[i]];
  area[v] = a;
}

dm_status mesh_areas(dm_ctx* ctx, MeshDev& m) {
  DArr<double> contrib;
  DM_ALLOC(ctx, contrib, size_t(m.nf) * 3);
  DM_ALLOC(ctx, m.area, size_t(m.nv));
  k_corner_area<<<grid_for(m.nf, 256), 256, 0, ctx->stream>>>(m.verts.p, m.faces.p, m.nf, contrib.p);
  k_vertex_area<<<grid_for(m.nv, 256), 256, 0, ctx->stream>>>(m.dkey.p, m.dval.p, int64_t(m.nf) * 3,
                                                              m.nv, contrib.p, m.area.p);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;   // contrib is freed in stream order
}

extern "C" dm_status dm_mixed_areas(dm_ctx* ctx, const dm_mesh* M, double* out) {
  if (!ctx || !M || !out) return DM_ERR_INVALID_ARG;
  DM_HIP(ctx, hipSetDevice(ctx->device));
  MeshDev tmp;
  DM_TRY(mesh_ingest(ctx, M, tmp, "A"));
  DM_TRY(mesh_areas(ctx, tmp));
  DM_HIP(ctx, hipMemcpyAsync(out, tmp.area.p, sizeof(double) * tmp.nv, hipMemcpyDeviceToDevice,
                             ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DM_OK;
}
