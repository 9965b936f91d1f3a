// ORACLE -- test infrastructure only.
//
// A plain, slow, single-threaded FP64 CPU implementation of the geometrically
// consistent product-triangle ILP and of its Jacobi min-marginal-averaging dual
// solver.  It exists to check the HIP library: only the tests, the smoke check
// and the benchmark's CPU-baseline leg may load it.  It shares no code, header,
// table or helper with the library; the two only see the same seeded inputs.
//
// Every function follows a passage of the paper (arXiv 2310.08230):
//   * Sec. 3.1, Eq. (P)   product space, constraints A x = b, x binary;
//   * Sec. 3.2, Eq. (D)   Lagrangean decomposition, one subproblem per row;
//   * Appendix "Coarse-to-fine solving strategy", min-marginal equation;
//   * Sec. 4.2, Eq. (cost) costs from mixed areas and feature distances;
//   * Sec. 5 "Metrics"    primal-dual gap;
//   * Sec. 4.1, Alg. 1 and Appendix "Quasi-Newton Updates": L-BFGS steps
//     interleaved with MMA (two-loop direction, FindStepSize, history).
// Where the paper is silent (product-space conventions it defers to earlier
// work, the MMA schedule it defers to FastDOG, the rounding heuristic, the
// smoothed dual) the reading taken is written next to the code.
//
// Build: g++ -O2 -ffp-contract=off -std=c++17 -shared -fPIC (see build.py).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <utility>
#include <vector>

namespace {

constexpr int OK = 0;
constexpr int E_ARG = -1;
constexpr int E_MESH = -2;
constexpr int E_GENUS = -3;
constexpr int E_INFEASIBLE = -4;
constexpr int E_NONFINITE = -5;

constexpr double INF = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Meshes (Table "notation": V in R^{|V| x 3}, T in N^{|T| x 3}).
// A valid input is a closed, oriented 2-manifold: every undirected edge lies in
// exactly two faces, traversed once in each direction, and the faces around
// every vertex form one cycle.  Edge ids are the ranks of the sorted (min, max)
// vertex pairs.  (Sec. 5 "Datasets": only watertight, same-genus pairs admit a
// solution of (P).)
// ---------------------------------------------------------------------------
struct Mesh {
  int nv = 0, nf = 0, ne = 0;
  std::vector<double> V;                 // nv*3
  std::vector<int> F;                    // nf*3
  std::vector<std::pair<int, int>> E;    // sorted (min, max)
  std::vector<int> FE;                   // nf*3: edge id of (F[k], F[k+1])
};

int edge_id(const Mesh& m, int a, int b) {
  std::pair<int, int> key(std::min(a, b), std::max(a, b));
  auto it = std::lower_bound(m.E.begin(), m.E.end(), key);
  if (it == m.E.end() || *it != key) return -1;
  return int(it - m.E.begin());
}

int mesh_build(Mesh& m, int nv, int nf, const float* verts, const int* faces) {
  if (nv <= 0 || nf <= 0 || !faces) return E_ARG;
  m.nv = nv;
  m.nf = nf;
  m.F.assign(faces, faces + 3 * nf);
  m.V.assign(3 * size_t(nv), 0.0);
  if (verts)
    for (size_t i = 0; i < 3 * size_t(nv); ++i) {
      if (!std::isfinite(verts[i])) return E_NONFINITE;
      m.V[i] = verts[i];
    }
  std::vector<int> used(nv, 0);
  std::vector<std::pair<int, int>> directed;
  for (int f = 0; f < nf; ++f) {
    const int* t = &m.F[3 * f];
    for (int k = 0; k < 3; ++k) {
      if (t[k] < 0 || t[k] >= nv) return E_MESH;
      used[t[k]] = 1;
    }
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) return E_MESH;
    for (int k = 0; k < 3; ++k) directed.emplace_back(t[k], t[(k + 1) % 3]);
  }
  for (int v = 0; v < nv; ++v)
    if (!used[v]) return E_MESH;
  // every directed edge once, and its reverse once
  std::sort(directed.begin(), directed.end());
  for (size_t i = 1; i < directed.size(); ++i)
    if (directed[i] == directed[i - 1]) return E_MESH;
  for (auto& d : directed)
    if (!std::binary_search(directed.begin(), directed.end(), std::make_pair(d.second, d.first)))
      return E_MESH;
  for (auto& d : directed)
    if (d.first < d.second) m.E.push_back(d);
  std::sort(m.E.begin(), m.E.end());
  m.ne = int(m.E.size());
  m.FE.resize(3 * size_t(nf));
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 3; ++k) m.FE[3 * f + k] = edge_id(m, m.F[3 * f + k], m.F[3 * f + (k + 1) % 3]);
  // vertex manifoldness: walking the fan around v (via "the face that holds
  // directed edge v->w") returns to its start after visiting every incident face
  std::vector<int> deg(nv, 0);
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 3; ++k) deg[m.F[3 * f + k]]++;
  // map directed edge -> face
  std::vector<std::pair<std::pair<int, int>, int>> dface;
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 3; ++k) dface.push_back({{m.F[3 * f + k], m.F[3 * f + (k + 1) % 3]}, f});
  std::sort(dface.begin(), dface.end());
  auto face_of = [&](int a, int b) {
    auto it = std::lower_bound(dface.begin(), dface.end(), std::make_pair(std::make_pair(a, b), -1));
    return it->second;
  };
  std::vector<int> start(nv, -1);
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 3; ++k)
      if (start[m.F[3 * f + k]] < 0) start[m.F[3 * f + k]] = f;
  for (int v = 0; v < nv; ++v) {
    int f = start[v], count = 0;
    do {
      const int* t = &m.F[3 * f];
      int k = (t[0] == v) ? 0 : (t[1] == v) ? 1 : 2;
      int prev = t[(k + 2) % 3];       // directed edge prev->v lies in f, so v->prev lies in the next face
      f = face_of(v, prev);
      ++count;
      if (count > deg[v]) return E_MESH;
    } while (f != start[v]);
    if (count != deg[v]) return E_MESH;
  }
  return OK;
}

// ---------------------------------------------------------------------------
// Mixed (Voronoi) vertex areas of Meyer et al. 2003, used as A^M, A^N in
// Eq. (cost) (Sec. 4.2).  Per triangle (p, q, r): if no angle is obtuse, p gets
// (|pq|^2 cot(r) + |pr|^2 cot(q)) / 8; if the angle at p is obtuse, area/2;
// if another angle is obtuse, area/4.
// ---------------------------------------------------------------------------
void mixed_areas(const Mesh& m, std::vector<double>& A) {
  A.assign(m.nv, 0.0);
  for (int f = 0; f < m.nf; ++f) {
    int id[3] = {m.F[3 * f], m.F[3 * f + 1], m.F[3 * f + 2]};
    double P[3][3];
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) P[k][c] = m.V[3 * size_t(id[k]) + c];
    auto sub = [](const double* a, const double* b, double* o) {
      for (int c = 0; c < 3; ++c) o[c] = a[c] - b[c];
    };
    auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    double e01[3], e02[3];
    sub(P[1], P[0], e01);
    sub(P[2], P[0], e02);
    double cr[3] = {e01[1] * e02[2] - e01[2] * e02[1], e01[2] * e02[0] - e01[0] * e02[2],
                    e01[0] * e02[1] - e01[1] * e02[0]};
    double area = 0.5 * std::sqrt(dot(cr, cr));
    double dots[3];  // dot product of the two edges leaving vertex k
    for (int k = 0; k < 3; ++k) {
      double u[3], w[3];
      sub(P[(k + 1) % 3], P[k], u);
      sub(P[(k + 2) % 3], P[k], w);
      dots[k] = dot(u, w);
    }
    bool obtuse = dots[0] < 0 || dots[1] < 0 || dots[2] < 0;
    for (int k = 0; k < 3; ++k) {
      double add;
      if (!obtuse) {
        int q = (k + 1) % 3, r = (k + 2) % 3;
        double pq[3], pr[3];
        sub(P[q], P[k], pq);
        sub(P[r], P[k], pr);
        // cot of the angle at r (opposite pq) and at q (opposite pr)
        double rq[3], rp[3], qr[3], qp[3];
        sub(P[q], P[r], rq);
        sub(P[k], P[r], rp);
        sub(P[r], P[q], qr);
        sub(P[k], P[q], qp);
        double twice_area = 2.0 * area;
        double cot_r = dot(rq, rp) / twice_area;
        double cot_q = dot(qr, qp) / twice_area;
        add = (dot(pq, pq) * cot_r + dot(pr, pr) * cot_q) / 8.0;
      } else if (dots[k] < 0) {
        add = area / 2.0;
      } else {
        add = area / 4.0;
      }
      A[id[k]] += add;
    }
  }
}

// ---------------------------------------------------------------------------
// Candidates.  The paper prunes product spaces only in its coarse-to-fine
// scheme and leaves the rule open; the reading used here: Euclidean
// descriptor distance in FP64, the K nearest in each direction (ties to the
// lower index), and the candidate set C is the union of both directions.
// ---------------------------------------------------------------------------
double desc_dist(const float* a, const float* b, int D) {
  double s = 0.0;
  for (int k = 0; k < D; ++k) {
    double d = double(a[k]) - double(b[k]);
    s += d * d;
  }
  return std::sqrt(s);
}

void knn(int na, const float* A, int nb, const float* B, int D, int K, int* out) {
  std::vector<std::pair<double, int>> row(nb);
  for (int i = 0; i < na; ++i) {
    for (int j = 0; j < nb; ++j) row[j] = {desc_dist(A + size_t(i) * D, B + size_t(j) * D, D), j};
    std::partial_sort(row.begin(), row.begin() + K, row.end());
    for (int k = 0; k < K; ++k) out[size_t(i) * K + k] = row[k].second;
  }
}

// ---------------------------------------------------------------------------
// Product space P (Sec. 3.1, Fig. "matching elements"): triangle-triangle,
// triangle-edge and triangle-vertex elements, in both directions.  The paper
// defers the exact element set to Windheuser et al. 2011; reading used here:
//   tri-tri    : X face (x1 x2 x3) as stored, Y face rotated by r = 0, 1, 2;
//   tri-edge   : X face, Y sequence on edge {b < b'} in the 6 patterns
//                (b b b') (b b' b) (b' b b) (b' b' b) (b' b b') (b b' b');
//   tri-vertex : X face, Y sequence (n n n);
//   edge-tri, vertex-tri : the same with the roles swapped (Y face as stored).
// A product vertex is (m, n) with id m * |V_Y| + n; an element is kept only
// if its three product vertices are candidate pairs.  Canonical order is the
// enumeration order: X class (face < edge < vertex), X id, Y class, Y id,
// rotation/pattern.
// ---------------------------------------------------------------------------
enum { CLS_FACE = 0, CLS_EDGE = 1, CLS_VERT = 2 };

void two_symbol_pattern(int pat, int b, int bp, int out[3]) {
  static const int P[6][3] = {{0, 0, 1}, {0, 1, 0}, {1, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
  for (int k = 0; k < 3; ++k) out[k] = P[pat][k] ? bp : b;
}

struct Space {
  Mesh X, Y;
  int K = 0;
  std::vector<uint8_t> cand;           // |V_X| * |V_Y|: 1 if (m, n) in C
  // product triangles
  std::vector<int> pv;                 // 3 per element
  std::vector<int> xid, yid;           // element ids within their class
  std::vector<uint8_t> xcls, ycls, pat;
  int64_t nP = 0;
  // full incidence A x = b (Eq. (P)): rows [closedness | X projection | Y projection]
  int64_t n_closed = 0, n_rows = 0;
  std::vector<int64_t> row_key;        // closedness: min * NPV + max; projection: face id
  std::vector<int64_t> row_ptr;
  std::vector<int64_t> ent_var;
  std::vector<int> ent_coef;
  std::vector<int> row_b;
  // presolve
  std::vector<int8_t> state;           // -1 free, 0 / 1 fixed
  // reduced problem on the free variables
  std::vector<int64_t> free_var;       // reduced var -> element
  std::vector<int64_t> var_red;        // element -> reduced var or -1
  std::vector<int64_t> rrow_orig;      // reduced row -> full row
  std::vector<int64_t> rrow_ptr;
  std::vector<int64_t> rent_var;
  std::vector<int> rent_coef;
  std::vector<int> rrow_b;
  std::vector<int> deg;                // reduced var -> number of reduced rows
  std::vector<std::vector<int64_t>> var_ents;  // reduced var -> its entries, ascending row
  // costs
  std::vector<double> cost;            // per element
  double offset = 0.0;
  bool has_cost = false;
};

int build_space(Space& S, const int* cand_xy, const int* cand_yx, int K) {
  const Mesh& X = S.X;
  const Mesh& Y = S.Y;
  const int64_t NVY = Y.nv;
  S.K = K;
  S.cand.assign(size_t(X.nv) * Y.nv, 0);
  for (int m = 0; m < X.nv; ++m)
    for (int k = 0; k < K; ++k) {
      int n = cand_xy[size_t(m) * K + k];
      if (n < 0 || n >= Y.nv) return E_ARG;
      S.cand[size_t(m) * NVY + n] = 1;
    }
  for (int n = 0; n < Y.nv; ++n)
    for (int k = 0; k < K; ++k) {
      int m = cand_yx[size_t(n) * K + k];
      if (m < 0 || m >= X.nv) return E_ARG;
      S.cand[size_t(m) * NVY + n] = 1;
    }
  auto emit = [&](const int xs[3], const int ys[3], int xc, int xi, int yc, int yi, int p) {
    for (int k = 0; k < 3; ++k)
      if (!S.cand[size_t(xs[k]) * NVY + ys[k]]) return;
    for (int k = 0; k < 3; ++k) S.pv.push_back(int(xs[k] * NVY + ys[k]));
    S.xcls.push_back(uint8_t(xc));
    S.xid.push_back(xi);
    S.ycls.push_back(uint8_t(yc));
    S.yid.push_back(yi);
    S.pat.push_back(uint8_t(p));
  };
  int xs[3], ys[3];
  for (int f = 0; f < X.nf; ++f) {
    for (int k = 0; k < 3; ++k) xs[k] = X.F[3 * f + k];
    for (int g = 0; g < Y.nf; ++g)
      for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) ys[k] = Y.F[3 * g + (k + r) % 3];
        emit(xs, ys, CLS_FACE, f, CLS_FACE, g, r);
      }
    for (int e = 0; e < Y.ne; ++e)
      for (int p = 0; p < 6; ++p) {
        two_symbol_pattern(p, Y.E[e].first, Y.E[e].second, ys);
        emit(xs, ys, CLS_FACE, f, CLS_EDGE, e, p);
      }
    for (int n = 0; n < Y.nv; ++n) {
      ys[0] = ys[1] = ys[2] = n;
      emit(xs, ys, CLS_FACE, f, CLS_VERT, n, 0);
    }
  }
  for (int e = 0; e < X.ne; ++e)
    for (int g = 0; g < Y.nf; ++g)
      for (int p = 0; p < 6; ++p) {
        two_symbol_pattern(p, X.E[e].first, X.E[e].second, xs);
        for (int k = 0; k < 3; ++k) ys[k] = Y.F[3 * g + k];
        emit(xs, ys, CLS_EDGE, e, CLS_FACE, g, p);
      }
  for (int m = 0; m < X.nv; ++m)
    for (int g = 0; g < Y.nf; ++g) {
      xs[0] = xs[1] = xs[2] = m;
      for (int k = 0; k < 3; ++k) ys[k] = Y.F[3 * g + k];
      emit(xs, ys, CLS_VERT, m, CLS_FACE, g, 0);
    }
  S.nP = int64_t(S.xcls.size());

  // Constraints (Sec. 3.1, Eq. (P)).  Closedness A^d x = 0: one row per
  // undirected product edge; a triangle traversing it from the smaller to the
  // larger product-vertex id contributes +1, the other way -1.  Projection
  // A^M x = 1 / A^N x = 1: one row per face of each shape over the elements
  // whose X (resp. Y) side is that face.
  const int64_t NPV = int64_t(X.nv) * NVY;
  std::vector<std::pair<int64_t, int64_t>> keyed;   // (key, element*3+k)
  keyed.reserve(size_t(3 * S.nP));
  for (int64_t p = 0; p < S.nP; ++p)
    for (int k = 0; k < 3; ++k) {
      int64_t a = S.pv[3 * p + k], b = S.pv[3 * p + (k + 1) % 3];
      keyed.emplace_back(std::min(a, b) * NPV + std::max(a, b), 3 * p + k);
    }
  std::sort(keyed.begin(), keyed.end());
  S.row_ptr.clear();
  S.row_key.clear();
  S.ent_var.clear();
  S.ent_coef.clear();
  S.row_b.clear();
  for (size_t i = 0; i < keyed.size(); ++i) {
    if (i == 0 || keyed[i].first != keyed[i - 1].first) {
      S.row_ptr.push_back(int64_t(S.ent_var.size()));
      S.row_key.push_back(keyed[i].first);
      S.row_b.push_back(0);
    }
    int64_t p = keyed[i].second / 3;
    int k = int(keyed[i].second % 3);
    int64_t a = S.pv[3 * p + k], b = S.pv[3 * p + (k + 1) % 3];
    S.ent_var.push_back(p);
    S.ent_coef.push_back(a < b ? +1 : -1);
  }
  S.n_closed = int64_t(S.row_key.size());
  std::vector<std::vector<int64_t>> xrows(X.nf), yrows(Y.nf);
  for (int64_t p = 0; p < S.nP; ++p) {
    if (S.xcls[p] == CLS_FACE) xrows[S.xid[p]].push_back(p);
    if (S.ycls[p] == CLS_FACE) yrows[S.yid[p]].push_back(p);
  }
  for (int f = 0; f < X.nf; ++f) {
    S.row_ptr.push_back(int64_t(S.ent_var.size()));
    S.row_key.push_back(f);
    S.row_b.push_back(1);
    for (int64_t p : xrows[f]) {
      S.ent_var.push_back(p);
      S.ent_coef.push_back(1);
    }
  }
  for (int g = 0; g < Y.nf; ++g) {
    S.row_ptr.push_back(int64_t(S.ent_var.size()));
    S.row_key.push_back(g);
    S.row_b.push_back(1);
    for (int64_t p : yrows[g]) {
      S.ent_var.push_back(p);
      S.ent_coef.push_back(1);
    }
  }
  S.row_ptr.push_back(int64_t(S.ent_var.size()));
  S.n_rows = int64_t(S.row_b.size());
  return OK;
}

// ---------------------------------------------------------------------------
// Presolve (not in the paper; needed so that every subproblem of Eq. (D) has
// finite min-marginals once pruning leaves one-sided rows).  Integer unit
// propagation to a fixpoint: in a row with residual r = b - sum(a x over
// variables fixed to 1) and P (N) free +1 (-1) entries, x_i = 1 (or 0) is
// excluded when the rest of the row can no longer reach the residual.  Rows
// whose entries are all fixed are dropped; a row whose residual lies outside
// [-N, P] proves the ILP infeasible.
// ---------------------------------------------------------------------------
// fix: optional starting assignment per element (-1 free, 0 / 1 fixed), the
// confident-variable fixing of the coarse-to-fine appendix
int presolve(Space& S, const int8_t* fix = nullptr) {
  S.state.assign(size_t(S.nP), -1);
  if (fix)
    for (int64_t p = 0; p < S.nP; ++p) S.state[p] = fix[p] < 0 ? int8_t(-1) : int8_t(fix[p] ? 1 : 0);
  bool changed = true;
  while (changed) {
    changed = false;
    for (int64_t j = 0; j < S.n_rows; ++j) {
      int64_t r = S.row_b[j];
      int64_t P = 0, N = 0;
      for (int64_t e = S.row_ptr[j]; e < S.row_ptr[j + 1]; ++e) {
        int8_t s = S.state[S.ent_var[e]];
        if (s == 1) r -= S.ent_coef[e];
        else if (s < 0) (S.ent_coef[e] > 0 ? P : N)++;
      }
      if (r < -N || r > P) return E_INFEASIBLE;
      for (int64_t e = S.row_ptr[j]; e < S.row_ptr[j + 1]; ++e) {
        int64_t v = S.ent_var[e];
        if (S.state[v] >= 0) continue;
        int a = S.ent_coef[e];
        // rest of the row without this entry
        int64_t Pr = P - (a > 0), Nr = N - (a < 0);
        bool one_ok = (r - a >= -Nr) && (r - a <= Pr);
        bool zero_ok = (r >= -Nr) && (r <= Pr);
        if (!one_ok && !zero_ok) return E_INFEASIBLE;
        if (!one_ok || !zero_ok) {
          S.state[v] = one_ok ? 1 : 0;
          changed = true;
          // the row's counts changed: recompute from scratch for the rest
          r = S.row_b[j];
          P = N = 0;
          for (int64_t e2 = S.row_ptr[j]; e2 < S.row_ptr[j + 1]; ++e2) {
            int8_t s2 = S.state[S.ent_var[e2]];
            if (s2 == 1) r -= S.ent_coef[e2];
            else if (s2 < 0) (S.ent_coef[e2] > 0 ? P : N)++;
          }
          if (r < -N || r > P) return E_INFEASIBLE;
        }
      }
    }
  }
  // reduced problem
  S.var_red.assign(size_t(S.nP), -1);
  S.free_var.clear();
  for (int64_t p = 0; p < S.nP; ++p)
    if (S.state[p] < 0) {
      S.var_red[p] = int64_t(S.free_var.size());
      S.free_var.push_back(p);
    }
  S.rrow_orig.clear();
  S.rrow_ptr.clear();
  S.rent_var.clear();
  S.rent_coef.clear();
  S.rrow_b.clear();
  for (int64_t j = 0; j < S.n_rows; ++j) {
    int64_t r = S.row_b[j], nfree = 0;
    for (int64_t e = S.row_ptr[j]; e < S.row_ptr[j + 1]; ++e) {
      int8_t s = S.state[S.ent_var[e]];
      if (s == 1) r -= S.ent_coef[e];
      if (s < 0) ++nfree;
    }
    if (nfree == 0) {
      if (r != 0) return E_INFEASIBLE;
      continue;
    }
    S.rrow_orig.push_back(j);
    S.rrow_ptr.push_back(int64_t(S.rent_var.size()));
    S.rrow_b.push_back(int(r));
    for (int64_t e = S.row_ptr[j]; e < S.row_ptr[j + 1]; ++e)
      if (S.state[S.ent_var[e]] < 0) {
        S.rent_var.push_back(S.var_red[S.ent_var[e]]);
        S.rent_coef.push_back(S.ent_coef[e]);
      }
  }
  S.rrow_ptr.push_back(int64_t(S.rent_var.size()));
  const int64_t nfv = int64_t(S.free_var.size());
  S.deg.assign(size_t(nfv), 0);
  S.var_ents.assign(size_t(nfv), {});
  for (size_t j = 0; j + 1 < S.rrow_ptr.size(); ++j)
    for (int64_t e = S.rrow_ptr[j]; e < S.rrow_ptr[j + 1]; ++e) {
      S.deg[S.rent_var[e]]++;
      S.var_ents[S.rent_var[e]].push_back(e);
    }
  // a free variable in no remaining row can be set to 0 (c >= 0); with the
  // rows above this never happens, every element lies in three closedness rows
  for (int64_t i = 0; i < nfv; ++i)
    if (S.deg[i] == 0) return E_ARG;
  return OK;
}

// ---------------------------------------------------------------------------
// One subproblem S_j = {s in {0,1}^{I_j} : sum a_ji s_i = b_j} of Eq. (D).
// Its minimum and the min-marginal differences
//   M_i = min_{s in S_j, s_i = 1} s^T lam  -  min_{s in S_j, s_i = 0} s^T lam
// (Appendix "Coarse-to-fine", min-marginal equation) are computed by the
// shortest-path recursion over partial sums sigma (the BDD of the row,
// Sec. 4.1): F_l(sigma) over the first l entries, B_l(sigma) over the rest,
// restricted to sums from which b stays reachable.  With temperature T > 0 the
// min is replaced by the soft-min  -T log sum exp(-./T)  (smoothed dual), and
// mu_i = P(s_i = 1) is returned as well.
// ---------------------------------------------------------------------------
struct RowOut {
  double rowmin;
};

inline double smin2(double a, double b, double T) {
  if (T <= 0.0) return std::min(a, b);
  if (a == INF) return b;
  if (b == INF) return a;
  double m = std::min(a, b);
  return m - T * std::log(std::exp(-(a - m) / T) + std::exp(-(b - m) / T));
}

double row_dp(int n, const int* a, int b, const double* lam, double T, double* M, double* mu) {
  // prefix counts and the reachable band of partial sums after l entries
  std::vector<int> Pp(n + 1, 0), Np(n + 1, 0);
  for (int l = 0; l < n; ++l) {
    Pp[l + 1] = Pp[l] + (a[l] > 0);
    Np[l + 1] = Np[l] + (a[l] < 0);
  }
  const int Pt = Pp[n], Nt = Np[n];
  std::vector<int> lo(n + 1), hi(n + 1);
  for (int l = 0; l <= n; ++l) {
    int Prest = Pt - Pp[l], Nrest = Nt - Np[l];
    lo[l] = std::max(-Np[l], b - Prest);
    hi[l] = std::min(Pp[l], b + Nrest);
  }
  std::vector<std::vector<double>> Fv(n + 1), Bv(n + 1);
  auto at = [&](std::vector<std::vector<double>>& tab, int l, int s) -> double {
    if (s < lo[l] || s > hi[l]) return INF;
    return tab[l][s - lo[l]];
  };
  for (int l = 0; l <= n; ++l) {
    Fv[l].assign(std::max(0, hi[l] - lo[l] + 1), INF);
    Bv[l].assign(std::max(0, hi[l] - lo[l] + 1), INF);
  }
  if (lo[0] <= 0 && 0 <= hi[0]) Fv[0][0 - lo[0]] = 0.0;
  for (int l = 0; l < n; ++l)
    for (int s = lo[l + 1]; s <= hi[l + 1]; ++s)
      Fv[l + 1][s - lo[l + 1]] = smin2(at(Fv, l, s), at(Fv, l, s - a[l]) + lam[l], T);
  if (lo[n] <= b && b <= hi[n]) Bv[n][b - lo[n]] = 0.0;
  for (int l = n - 1; l >= 0; --l)
    for (int s = lo[l]; s <= hi[l]; ++s)
      Bv[l][s - lo[l]] = smin2(at(Bv, l + 1, s), at(Bv, l + 1, s + a[l]) + lam[l], T);
  const double total = at(Bv, 0, 0);
  for (int l = 0; l < n; ++l) {
    double m1 = INF, m0 = INF;
    for (int s = lo[l]; s <= hi[l]; ++s) {
      double f = at(Fv, l, s);
      if (f == INF) continue;
      m1 = smin2(m1, f + lam[l] + at(Bv, l + 1, s + a[l]), T);
      m0 = smin2(m0, f + at(Bv, l + 1, s), T);
    }
    if (M) M[l] = m1 - m0;
    if (mu) mu[l] = (T > 0.0) ? std::exp(-(m1 - total) / T) : (m1 <= m0 ? 1.0 : 0.0);
  }
  return total;
}

// ---------------------------------------------------------------------------
// Dual (D): sum over rows of subproblem minima, plus the constant from the
// variables presolve fixed to 1.  Evaluated at one lambda snapshot.
// ---------------------------------------------------------------------------
double sweep(const Space& S, const double* lam, double T, double* M, double* rowmin, double* mu) {
  const int64_t nr = int64_t(S.rrow_b.size());
  double lb = S.offset;
  std::vector<double> rm(static_cast<size_t>(nr));
  for (int64_t j = 0; j < nr; ++j) {
    int64_t b0 = S.rrow_ptr[j], n = S.rrow_ptr[j + 1] - b0;
    rm[j] = row_dp(int(n), &S.rent_coef[b0], S.rrow_b[j], lam + b0, T, M ? M + b0 : nullptr,
                   mu ? mu + b0 : nullptr);
  }
  for (int64_t j = 0; j < nr; ++j) {
    lb += rm[j];
    if (rowmin) rowmin[j] = rm[j];
  }
  return lb;
}

// ---------------------------------------------------------------------------
// Min-marginal averaging (Sec. 3.2 and Alg. 1's MMA step, deferred to
// FastDOG).  The paper does not restate FastDOG's schedule; the reading used
// here is the fully parallel (Jacobi) form with damping omega:
//   M from every row at the snapshot lambda_t,
//   Mbar_i = mean of M^j_i over the rows J_i holding i,
//   lambda^j_i <- lambda^j_i - omega (M^j_i - Mbar_i),
// which keeps sum_j lambda^j_i = c_i (the constraint of Eq. (D)).  The trace
// holds the bound at lambda_t before each update.
// ---------------------------------------------------------------------------
void init_lambda(const Space& S, double* lam) {
  for (size_t i = 0; i < S.free_var.size(); ++i)
    for (int64_t e : S.var_ents[i]) lam[e] = S.cost[S.free_var[i]] / S.deg[i];
}

void jacobi(const Space& S, double* lam, int iters, double omega, double T, double* trace) {
  const int64_t nnz = int64_t(S.rent_var.size());
  std::vector<double> M(static_cast<size_t>(nnz));
  for (int t = 0; t < iters; ++t) {
    double lb = sweep(S, lam, T, M.data(), nullptr, nullptr);
    if (trace) trace[t] = lb;
    for (size_t i = 0; i < S.free_var.size(); ++i) {
      double sum = 0.0;
      for (int64_t e : S.var_ents[i]) sum += M[e];
      double mbar = sum / S.deg[i];
      for (int64_t e : S.var_ents[i]) lam[e] -= omega * (M[e] - mbar);
    }
  }
}

// ---------------------------------------------------------------------------
// Costs, Eq. (cost) (Sec. 4.2): c_p = sum_v (A_X(m_v) + A_Y(n_v)) ||F_X(m_v)
// - F_Y(n_v)|| over the three product vertices of p (a vertex pair repeated in
// a degenerate element counts each time).  The norm is read as Euclidean and
// unsquared; the areas are those of the posed meshes.
// ---------------------------------------------------------------------------
int compute_costs(Space& S, const float* DX, const float* DY, int D) {
  std::vector<double> AX, AY;
  mixed_areas(S.X, AX);
  mixed_areas(S.Y, AY);
  const int64_t NVY = S.Y.nv;
  S.cost.assign(size_t(S.nP), 0.0);
  for (int64_t p = 0; p < S.nP; ++p) {
    double c = 0.0;
    for (int k = 0; k < 3; ++k) {
      int64_t q = S.pv[3 * p + k];
      int m = int(q / NVY), n = int(q % NVY);
      c += (AX[m] + AY[n]) * desc_dist(DX + size_t(m) * D, DY + size_t(n) * D, D);
    }
    if (!std::isfinite(c)) return E_NONFINITE;
    S.cost[p] = c;
  }
  S.offset = 0.0;
  for (int64_t p = 0; p < S.nP; ++p)
    if (S.state[p] == 1) S.offset += S.cost[p];
  S.has_cost = true;
  return OK;
}

// counter-based generator: splitmix64 (Steele, Lea, Flood 2014) of a key built
// from (seed, round, variable); maps to a double in [-1, 1)
uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform_pm1(uint64_t seed, uint32_t round, uint32_t var) {
  uint64_t key = splitmix64(seed) ^ ((uint64_t(round) << 32) | uint64_t(var));
  uint64_t z = splitmix64(key);
  return double(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// exact integer check of A x = b over every row of the full ILP (Eq. (P))
int64_t violations(const Space& S, const uint8_t* x) {
  int64_t bad = 0;
  for (int64_t j = 0; j < S.n_rows; ++j) {
    int64_t s = 0;
    for (int64_t e = S.row_ptr[j]; e < S.row_ptr[j + 1]; ++e)
      if (x[S.ent_var[e]]) s += S.ent_coef[e];
    if (s != S.row_b[j]) ++bad;
  }
  return bad;
}

}  // namespace

// ===========================================================================
// C entry points (ctypes).
// ===========================================================================
extern "C" {

int or_mesh_check(int nv, int nf, const int* faces, int* n_edges) {
  Mesh m;
  int st = mesh_build(m, nv, nf, nullptr, faces);
  if (st == OK && n_edges) *n_edges = m.ne;
  return st;
}

int or_mesh_edges(int nv, int nf, const int* faces, int* edges, int* face_edge) {
  Mesh m;
  int st = mesh_build(m, nv, nf, nullptr, faces);
  if (st != OK) return st;
  for (int e = 0; e < m.ne; ++e) {
    edges[2 * e] = m.E[e].first;
    edges[2 * e + 1] = m.E[e].second;
  }
  std::copy(m.FE.begin(), m.FE.end(), face_edge);
  return OK;
}

int or_mixed_areas(int nv, int nf, const float* verts, const int* faces, double* out) {
  Mesh m;
  int st = mesh_build(m, nv, nf, verts, faces);
  if (st != OK) return st;
  std::vector<double> A;
  mixed_areas(m, A);
  std::copy(A.begin(), A.end(), out);
  return OK;
}

int or_knn(int nvx, const float* FX, int nvy, const float* FY, int D, int K, int* cand_xy,
           int* cand_yx) {
  if (K <= 0 || K > nvx || K > nvy || D <= 0) return E_ARG;
  for (size_t i = 0; i < size_t(nvx) * D; ++i)
    if (!std::isfinite(FX[i])) return E_NONFINITE;
  for (size_t i = 0; i < size_t(nvy) * D; ++i)
    if (!std::isfinite(FY[i])) return E_NONFINITE;
  knn(nvx, FX, nvy, FY, D, K, cand_xy);
  knn(nvy, FY, nvx, FX, D, K, cand_yx);
  return OK;
}

int or_desc_dist(int n, const int* m_idx, const int* n_idx, const float* FX, const float* FY, int D,
                 double* out) {
  for (int i = 0; i < n; ++i)
    out[i] = desc_dist(FX + size_t(m_idx[i]) * D, FY + size_t(n_idx[i]) * D, D);
  return OK;
}

void* or_space_build(int nvx, int nfx, const float* VX, const int* FX, int nvy, int nfy,
                     const float* VY, const int* FY, const int* cand_xy, const int* cand_yx, int K,
                     int* status) {
  Space* S = new Space();
  int st = mesh_build(S->X, nvx, nfx, VX, FX);
  if (st == OK) st = mesh_build(S->Y, nvy, nfy, VY, FY);
  if (st == OK && (S->X.nv - S->X.ne + S->X.nf) != (S->Y.nv - S->Y.ne + S->Y.nf)) st = E_GENUS;
  if (st == OK && (K <= 0 || K > nvx || K > nvy)) st = E_ARG;
  if (st == OK) st = build_space(*S, cand_xy, cand_yx, K);
  if (st == OK) st = presolve(*S);
  *status = st;
  if (st != OK) {
    delete S;
    return nullptr;
  }
  return S;
}

// Generic 0-1 ILP with +-1 rows (Appendix "Other ILPs": the solver is not
// specific to matching).  The decomposition of Eq. (D) as stated: one
// subproblem per input row, over the distinct variables of that row, and a
// variable's multipliers sum to its cost over the rows it lies in (1 to 5).
// Exactly-one rows (all +1, b = 1) keep any length, the others at most 64
// entries.  Row order: the other input rows, then the exactly-one input rows
// (each group in input order); a variable named twice in one row is
// rejected.
void* or_ilp_build(int n_vars, int n_rows, const int* row_ptr, const int* cols, const int* coefs, const int* b,
                   int* status) {
  *status = E_ARG;
  if (n_vars < 1 || n_rows < 0) return nullptr;
  std::vector<int> deg(size_t(n_vars), 0);
  std::vector<bool> exactly_one(size_t(n_rows), false);
  for (int j = 0; j < n_rows; ++j) {
    bool all_pos = true;
    std::vector<int> seen;
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
      if (coefs[e] != 1 && coefs[e] != -1) return nullptr;
      if (cols[e] < 0 || cols[e] >= n_vars) return nullptr;
      all_pos = all_pos && coefs[e] == 1;
      seen.push_back(cols[e]);
      ++deg[size_t(cols[e])];
    }
    std::sort(seen.begin(), seen.end());
    for (size_t i = 1; i < seen.size(); ++i)
      if (seen[i] == seen[i - 1]) return nullptr;   // a variable twice in one row
    const int len = row_ptr[j + 1] - row_ptr[j];
    exactly_one[size_t(j)] = all_pos && b[j] == 1 && len > 0;
    if (!exactly_one[size_t(j)] && len > 64) return nullptr;
  }
  for (int v = 0; v < n_vars; ++v)
    if (deg[size_t(v)] < 1 || deg[size_t(v)] > 5) return nullptr;
  Space* S = new Space();
  S->nP = n_vars;
  auto add_input_row = [&](int j) {
    S->row_key.push_back(j);
    S->row_b.push_back(b[j]);
    S->row_ptr.push_back(int64_t(S->ent_var.size()));
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
      S->ent_var.push_back(cols[e]);
      S->ent_coef.push_back(coefs[e]);
    }
  };
  for (int j = 0; j < n_rows; ++j)
    if (!exactly_one[size_t(j)]) add_input_row(j);
  S->n_closed = int64_t(S->row_b.size());
  for (int j = 0; j < n_rows; ++j)
    if (exactly_one[size_t(j)]) add_input_row(j);
  S->n_rows = int64_t(S->row_b.size());
  S->row_ptr.push_back(int64_t(S->ent_var.size()));
  const int st = presolve(*S);
  *status = st;
  if (st != OK) {
    delete S;
    return nullptr;
  }
  return S;
}

void or_space_free(void* h) { delete static_cast<Space*>(h); }

// info: [nP, n_rows_full, nnz_full, n_closed_full, n_free, n_fixed1, n_rows_red, nnz_red]
void or_space_info(void* h, int64_t* info) {
  Space& S = *static_cast<Space*>(h);
  int64_t nfix1 = 0;
  for (auto s : S.state) nfix1 += (s == 1);
  info[0] = S.nP;
  info[1] = S.n_rows;
  info[2] = int64_t(S.ent_var.size());
  info[3] = S.n_closed;
  info[4] = int64_t(S.free_var.size());
  info[5] = nfix1;
  info[6] = int64_t(S.rrow_b.size());
  info[7] = int64_t(S.rent_var.size());
}

// which: 0 pv int32[nP*3]; 1 code int32[nP*4] (xcls, xid, ycls*8+pat, yid);
//        2 state int8[nP]; 3 row_key int64[n_rows]; 4 row_ptr int64[n_rows+1];
//        5 ent_var int64[nnz]; 6 ent_coef int32[nnz]; 7 row_b int32[n_rows];
//        8 free_var int64[n_free]; 9 rrow_orig int64; 10 rrow_ptr int64; 11 rent_var int64;
//        12 rent_coef int32; 13 rrow_b int32; 14 deg int32[n_free]; 15 cost double[nP];
//        16 offset double[1]; 17 cand uint8[nvx*nvy]; 18 edges X int32; 19 edges Y int32
int or_space_get(void* h, int which, void* dst) {
  Space& S = *static_cast<Space*>(h);
  auto cp = [&](const auto& v) {
    std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    return OK;
  };
  switch (which) {
    case 0: return cp(S.pv);
    case 1: {
      int* o = static_cast<int*>(dst);
      for (int64_t p = 0; p < S.nP; ++p) {
        o[4 * p] = S.xcls[p];
        o[4 * p + 1] = S.xid[p];
        o[4 * p + 2] = S.ycls[p] * 8 + S.pat[p];
        o[4 * p + 3] = S.yid[p];
      }
      return OK;
    }
    case 2: return cp(S.state);
    case 3: return cp(S.row_key);
    case 4: return cp(S.row_ptr);
    case 5: return cp(S.ent_var);
    case 6: return cp(S.ent_coef);
    case 7: return cp(S.row_b);
    case 8: return cp(S.free_var);
    case 9: return cp(S.rrow_orig);
    case 10: return cp(S.rrow_ptr);
    case 11: return cp(S.rent_var);
    case 12: return cp(S.rent_coef);
    case 13: return cp(S.rrow_b);
    case 14: return cp(S.deg);
    case 15: return cp(S.cost);
    case 16: *static_cast<double*>(dst) = S.offset; return OK;
    case 17: return cp(S.cand);
    case 18: case 19: {
      const Mesh& m = which == 18 ? S.X : S.Y;
      int* o = static_cast<int*>(dst);
      for (int e = 0; e < m.ne; ++e) {
        o[2 * e] = m.E[e].first;
        o[2 * e + 1] = m.E[e].second;
      }
      return OK;
    }
  }
  return E_ARG;
}

int or_space_costs(void* h, const float* DX, const float* DY, int D) {
  Space& S = *static_cast<Space*>(h);
  for (size_t i = 0; i < size_t(S.X.nv) * D; ++i)
    if (!std::isfinite(DX[i])) return E_NONFINITE;
  for (size_t i = 0; i < size_t(S.Y.nv) * D; ++i)
    if (!std::isfinite(DY[i])) return E_NONFINITE;
  return compute_costs(S, DX, DY, D);
}

int or_space_set_costs(void* h, const double* cost) {
  Space& S = *static_cast<Space*>(h);
  S.cost.assign(cost, cost + S.nP);
  S.offset = 0.0;
  for (int64_t p = 0; p < S.nP; ++p)
    if (S.state[p] == 1) S.offset += S.cost[p];
  S.has_cost = true;
  return OK;
}

int or_init_lambda(void* h, double* lam) {
  Space& S = *static_cast<Space*>(h);
  if (!S.has_cost) return E_ARG;
  init_lambda(S, lam);
  return OK;
}

int or_dual_solve(void* h, int iters, double omega, double T, double* lam, double* trace, int init) {
  Space& S = *static_cast<Space*>(h);
  if (!S.has_cost || iters < 0) return E_ARG;
  if (init) init_lambda(S, lam);
  jacobi(S, lam, iters, omega, T, trace);
  return OK;
}

double or_lower_bound(void* h, const double* lam, double T) {
  Space& S = *static_cast<Space*>(h);
  return sweep(S, lam, T, nullptr, nullptr, nullptr);
}

int or_min_marginals(void* h, const double* lam, double T, double* M, double* rowmin, double* mu) {
  Space& S = *static_cast<Space*>(h);
  sweep(S, lam, T, M, rowmin, mu);
  return OK;
}

double or_row_dp(int n, const int* coef, int b, const double* lam, double T, double* M, double* mu) {
  return row_dp(n, coef, b, lam, T, M, mu);
}

int64_t or_check_primal(void* h, const uint8_t* x) {
  return violations(*static_cast<Space*>(h), x);
}

// ---------------------------------------------------------------------------
// Primal rounding.  The paper uses FastDOG's heuristic driven by its own dual
// (Sec. 4, Fig. "pipeline"; Sec. 5 "Methods") without restating it.  Reading
// used here, built on the sign semantics of min-marginal differences
// (Appendix "Coarse-to-fine": M > 0 prefers 0, M < 0 prefers 1, a variable
// agrees when all its rows share the sign):
//   on a copy (c~, lam~), for r = 0..R: sweep all rows; if every free
//   variable agrees, x = the agreed assignment, checked exactly; else perturb
//   c~_i by Delta_i (-delta for agreed-1, +delta for agreed-0, delta u_i with
//   u_i in [-1, 1) from splitmix64(seed, r, i) otherwise), spread Delta_i /
//   deg(i) over lam~^j_i, run T_iters Jacobi iterations, delta *= gamma.
//   delta_0 <= 0 means 0.1 * mean |M| at the first sweep.
// ---------------------------------------------------------------------------
int or_round(void* h, const double* lam_in, int R, int T_iters, double delta0, double gamma,
             uint64_t seed, double omega, uint8_t* x, double* pobj, int* feasible, int* rounds) {
  Space& S = *static_cast<Space*>(h);
  if (!S.has_cost) return E_ARG;
  const int64_t nnz = int64_t(S.rent_var.size());
  const int64_t nfv = int64_t(S.free_var.size());
  std::vector<double> lam(lam_in, lam_in + nnz), M(static_cast<size_t>(nnz));
  double delta = delta0;
  *feasible = 0;
  for (int r = 0; r <= R; ++r) {
    sweep(S, lam.data(), 0.0, M.data(), nullptr, nullptr);
    if (r == 0 && delta <= 0.0) {
      double s = 0.0;
      for (int64_t e = 0; e < nnz; ++e) s += std::fabs(M[e]);
      delta = nnz ? 0.1 * s / double(nnz) : 0.0;
    }
    std::vector<int8_t> pref(size_t(nfv), -1);   // 1, 0 or -1 (no agreement)
    bool all = true;
    for (int64_t i = 0; i < nfv; ++i) {
      bool neg = true, pos = true;
      for (int64_t e : S.var_ents[i]) {
        neg = neg && (M[e] < 0.0);
        pos = pos && (M[e] > 0.0);
      }
      pref[i] = neg ? 1 : (pos ? 0 : -1);
      all = all && pref[i] >= 0;
    }
    for (int64_t p = 0; p < S.nP; ++p) x[p] = S.state[p] == 1 ? 1 : 0;
    for (int64_t i = 0; i < nfv; ++i) x[S.free_var[i]] = pref[i] == 1 ? 1 : 0;
    *rounds = r;
    if (all && violations(S, x) == 0) {
      *feasible = 1;
      break;
    }
    if (r == R) break;
    for (int64_t i = 0; i < nfv; ++i) {
      double d = pref[i] == 1 ? -delta : pref[i] == 0 ? delta
                                                      : delta * uniform_pm1(seed, uint32_t(r), uint32_t(i));
      for (int64_t e : S.var_ents[i]) lam[e] += d / S.deg[i];
    }
    jacobi(S, lam.data(), T_iters, omega, 0.0, nullptr);
    delta *= gamma;
  }
  double p = 0.0;
  for (int64_t q = 0; q < S.nP; ++q)
    if (x[q]) p += S.cost[q];
  *pobj = p;
  return OK;
}

double or_uniform_pm1(uint64_t seed, uint32_t round, uint32_t var) { return uniform_pm1(seed, round, var); }

// ---------------------------------------------------------------------------
// Smoothed dual and its gradient (not in the paper; the differentiable form
// of this library).  L_T(lam) = offset + sum_j softmin_T over S_j.  With
// lam^j_i = c_i / deg(i) + phi^j_i and phi held fixed,
//   dL/dc_i = mean over j of mu^j_i (free), 1 (fixed to 1), 0 (fixed to 0);
//   dL/dw(m, n) = sum of dL/dc_p over the product vertices (m, n) of p;
//   dL/dF_X(m) = sum_n dL/dw(m, n) (A_X(m) + A_Y(n)) (F_X(m) - F_Y(n)) / d(m, n)
// and the negative of the same terms for F_Y(n) (0 where d = 0).  Areas and
// candidates are constants.
// ---------------------------------------------------------------------------
int or_smoothed_grad(void* h, const double* lam, double T, const float* DX, const float* DY, int D,
                     double* gcost, double* gFX, double* gFY, double* value) {
  Space& S = *static_cast<Space*>(h);
  if (T <= 0.0 || !S.has_cost) return E_ARG;
  const int64_t nnz = int64_t(S.rent_var.size());
  std::vector<double> mu(static_cast<size_t>(nnz));
  double v = sweep(S, lam, T, nullptr, nullptr, mu.data());
  if (value) *value = v;
  std::vector<double> gc(size_t(S.nP), 0.0);
  for (int64_t p = 0; p < S.nP; ++p)
    if (S.state[p] == 1) gc[p] = 1.0;
  for (size_t i = 0; i < S.free_var.size(); ++i) {
    double s = 0.0;
    for (int64_t e : S.var_ents[i]) s += mu[e];
    gc[S.free_var[i]] = s / S.deg[i];
  }
  if (gcost) std::copy(gc.begin(), gc.end(), gcost);
  std::vector<double> AX, AY;
  mixed_areas(S.X, AX);
  mixed_areas(S.Y, AY);
  const int64_t NVY = S.Y.nv;
  std::fill(gFX, gFX + size_t(S.X.nv) * D, 0.0);
  std::fill(gFY, gFY + size_t(S.Y.nv) * D, 0.0);
  // dL/dw accumulated per product vertex
  std::vector<double> gw(size_t(S.X.nv) * NVY, 0.0);
  for (int64_t p = 0; p < S.nP; ++p)
    for (int k = 0; k < 3; ++k) gw[S.pv[3 * p + k]] += gc[p];
  for (int m = 0; m < S.X.nv; ++m)
    for (int n = 0; n < S.Y.nv; ++n) {
      double g = gw[size_t(m) * NVY + n];
      if (g == 0.0) continue;
      const float* a = DX + size_t(m) * D;
      const float* b = DY + size_t(n) * D;
      double d = desc_dist(a, b, D);
      if (d == 0.0) continue;
      double coef = g * (AX[m] + AY[n]) / d;
      for (int k = 0; k < D; ++k) {
        double diff = double(a[k]) - double(b[k]);
        gFX[size_t(m) * D + k] += coef * diff;
        gFY[size_t(n) * D + k] -= coef * diff;
      }
    }
  return OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Quasi-Newton powered MMA (Sec. 4.1, Alg. 1; Appendix "Quasi-Newton updates":
// the inverse-Hessian update, the L-BFGS direction and FindStepSize).
// One iteration: subgradient g (every row's minimising assignment), direction
// d^ = H g by the two-loop recursion, dual-feasible projection of d^, step size
// search, step, one MMA (Jacobi) iteration, history update.  Readings:
//   * L-BFGS is applied to the convex function -E, so the stored pairs are
//     s = lambda_{k+1} - lambda_k and y = g(lambda_k) - g(lambda_{k+1}) and
//     the curvature test s^T y >= eps keeps only pairs of positive curvature;
//   * with an empty history H = I; otherwise H0 = (s^T y / y^T y) I from the
//     newest pair, then the two-loop recursion;
//   * FindStepSize compares against E(lambda) (the objective before the step,
//     as the prose describes); Delta_min = 1e-6 (E(lambda^1) - E(lambda^0)),
//     +inf during the first invocation; the step is taken only if the best
//     trial improves on E(lambda);
//   * every row's minimiser takes ties to the lowest index (exactly-one rows)
//     or, for +-1 rows, the smallest count k of +1 entries and the entries of
//     lowest rank within each sign (rank by value, ties by position).
// ---------------------------------------------------------------------------
void row_argmin(int n, const int* a, int b, const double* lam, double* g) {
  // choose k entries of +1 and k - b of -1, each the cheapest of its sign
  std::vector<int> pos, neg;
  for (int l = 0; l < n; ++l) (a[l] > 0 ? pos : neg).push_back(l);
  auto by_value = [&](int x, int y) { return lam[x] < lam[y] || (lam[x] == lam[y] && x < y); };
  std::sort(pos.begin(), pos.end(), by_value);
  std::sort(neg.begin(), neg.end(), by_value);
  const int P = int(pos.size()), N = int(neg.size());
  double best = INF;
  int kbest = -1;
  for (int k = std::max(0, b); k <= std::min(P, N + b); ++k) {
    double f = 0.0;
    for (int q = 0; q < k; ++q) f += lam[pos[q]];
    for (int q = 0; q < k - b; ++q) f += lam[neg[q]];
    if (f < best) {
      best = f;
      kbest = k;
    }
  }
  for (int l = 0; l < n; ++l) g[l] = 0.0;
  for (int q = 0; q < kbest; ++q) g[pos[q]] = 1.0;
  for (int q = 0; q < kbest - b; ++q) g[neg[q]] = 1.0;
}

void subgradient(const Space& S, const double* lam, double* g) {
  const int64_t nr = int64_t(S.rrow_b.size());
  for (int64_t j = 0; j < nr; ++j) {
    int64_t b0 = S.rrow_ptr[j], n = S.rrow_ptr[j + 1] - b0;
    row_argmin(int(n), &S.rent_coef[b0], S.rrow_b[j], lam + b0, g + b0);
  }
}

// subtract from every multiplier direction the mean over its variable's rows
void project_feasible(const Space& S, double* d) {
  for (size_t i = 0; i < S.free_var.size(); ++i) {
    double sum = 0.0;
    for (int64_t e : S.var_ents[i]) sum += d[e];
    double mean = sum / S.deg[i];
    for (int64_t e : S.var_ents[i]) d[e] -= mean;
  }
}

double dotv(const std::vector<double>& x, const std::vector<double>& y) {
  double s = 0.0;
  for (size_t i = 0; i < x.size(); ++i) s += x[i] * y[i];
  return s;
}

// two-loop recursion: d = H g with history pairs (oldest first)
void lbfgs_direction(const std::vector<std::vector<double>>& Sh, const std::vector<std::vector<double>>& Yh,
                     const std::vector<double>& g, std::vector<double>& d) {
  const size_t m = Sh.size();
  d = g;
  if (m == 0) return;
  std::vector<double> alpha(m), rho(m);
  for (size_t j = m; j-- > 0;) {
    rho[j] = 1.0 / dotv(Sh[j], Yh[j]);
    alpha[j] = rho[j] * dotv(Sh[j], d);
    for (size_t e = 0; e < d.size(); ++e) d[e] -= alpha[j] * Yh[j][e];
  }
  const double h0 = dotv(Sh[m - 1], Yh[m - 1]) / dotv(Yh[m - 1], Yh[m - 1]);
  for (double& v : d) v *= h0;
  for (size_t j = 0; j < m; ++j) {
    const double beta = rho[j] * dotv(Yh[j], d);
    for (size_t e = 0; e < d.size(); ++e) d[e] += Sh[j][e] * (alpha[j] - beta);
  }
}

struct StepResult {
  double gamma, E_best;
};

// FindStepSize: grow gamma by a_up while the step does not reach Delta_min,
// shrink by a_down while it does not improve; keep the best trial
template <typename F>
StepResult find_step(F&& E_at, double E_init, double gamma, int K, double a_up, double a_down, double dmin) {
  double gm = gamma, Em = E_at(gamma), Ecur = Em;
  for (int t = 0; t < K; ++t) {
    gamma = (Ecur <= E_init) ? a_down * gamma : a_up * gamma;
    Ecur = E_at(gamma);
    if (Ecur >= Em) {
      gm = gamma;
      Em = Ecur;
    }
    if (Ecur - E_init >= dmin) break;
  }
  return {gm, Em};
}

}  // namespace

extern "C" {

int or_lbfgs_solve(void* h, int iters, double omega, int m, int K, double eps, double a_up, double a_down,
                   double gamma0, double* lam, double* trace_E, double* trace_gamma, int* taken) {
  Space& S = *static_cast<Space*>(h);
  if (!S.has_cost || iters < 0 || m < 0 || K < 1) return E_ARG;
  const size_t nnz = S.rent_var.size();
  std::vector<double> L(lam, lam + nnz), g(nnz), g_new(nnz), d(nnz), trial(nnz), L_prev(nnz);
  std::vector<std::vector<double>> Sh, Yh;
  double gamma = gamma0, dmin = INF, E0 = 0.0;
  double E_now = sweep(S, L.data(), 0.0, nullptr, nullptr, nullptr);
  subgradient(S, L.data(), g.data());
  for (int t = 0; t < iters; ++t) {
    if (trace_E) trace_E[t] = E_now;
    if (t == 0) E0 = E_now;
    if (t == 1) dmin = 1e-6 * (E_now - E0);
    lbfgs_direction(Sh, Yh, g, d);
    project_feasible(S, d.data());
    auto E_at = [&](double gm) {
      for (size_t e = 0; e < nnz; ++e) trial[e] = L[e] + gm * d[e];
      return sweep(S, trial.data(), 0.0, nullptr, nullptr, nullptr);
    };
    StepResult st = find_step(E_at, E_now, gamma, K, a_up, a_down, dmin);
    L_prev = L;
    gamma = st.gamma;
    if (trace_gamma) trace_gamma[t] = gamma;
    const bool step = st.E_best > E_now;
    if (taken) taken[t] = step ? 1 : 0;
    if (step)
      for (size_t e = 0; e < nnz; ++e) L[e] += gamma * d[e];
    jacobi(S, L.data(), 1, omega, 0.0, nullptr);
    E_now = sweep(S, L.data(), 0.0, nullptr, nullptr, nullptr);
    subgradient(S, L.data(), g_new.data());
    std::vector<double> s(nnz), y(nnz);
    for (size_t e = 0; e < nnz; ++e) {
      s[e] = L[e] - L_prev[e];
      y[e] = g[e] - g_new[e];
    }
    if (dotv(s, y) >= eps) {
      Sh.push_back(std::move(s));
      Yh.push_back(std::move(y));
      if (int(Sh.size()) > m) {
        Sh.erase(Sh.begin());
        Yh.erase(Yh.begin());
      }
    }
    g.swap(g_new);
  }
  if (trace_E) trace_E[iters] = E_now;
  std::copy(L.begin(), L.end(), lam);
  return OK;
}

// Confident-variable fixing (Appendix "Coarse-to-fine solving strategy"): at
// lambda, the min-marginal differences M^j_i of every free variable; a
// variable agrees when all its M^j_i are < 0 (prefers 1) or all > 0 (prefers
// 0); the agreeing variables are ranked by |sum_j M^j_i| (sum over its rows in
// ascending row order; ties to the lower variable) and the top
// floor(frac * count) are fixed to their preferred values.  fix[p] gets the
// presolve state of fixed elements, the new fixings, and -1 elsewhere.
// Returns the number of newly fixed variables in *n_fixed and the number of
// agreeing ones in *n_agree.
int or_confident_fix(void* h, const double* lam, double frac, int8_t* fix, int64_t* n_agree, int64_t* n_fixed) {
  Space& S = *static_cast<Space*>(h);
  if (!S.has_cost || !(frac >= 0.0 && frac <= 1.0)) return E_ARG;
  const size_t nnz = S.rent_var.size();
  std::vector<double> M(nnz);
  sweep(S, lam, 0.0, M.data(), nullptr, nullptr);
  struct Cand {
    double score;
    int64_t var;
    int8_t value;
  };
  std::vector<Cand> agree;
  for (size_t i = 0; i < S.free_var.size(); ++i) {
    bool neg = true, pos = true;
    double sum = 0.0;
    for (int64_t e : S.var_ents[i]) {
      neg = neg && M[e] < 0.0;
      pos = pos && M[e] > 0.0;
      sum += M[e];
    }
    if (neg || pos) agree.push_back({std::fabs(sum), int64_t(i), int8_t(neg ? 1 : 0)});
  }
  std::sort(agree.begin(), agree.end(), [](const Cand& a, const Cand& b) {
    return a.score > b.score || (a.score == b.score && a.var < b.var);
  });
  const size_t take = size_t(std::floor(frac * double(agree.size())));
  for (int64_t p = 0; p < S.nP; ++p) fix[p] = S.state[p];
  for (size_t k = 0; k < take; ++k) fix[S.free_var[agree[k].var]] = agree[k].value;
  if (n_agree) *n_agree = int64_t(agree.size());
  if (n_fixed) *n_fixed = int64_t(take);
  return OK;
}

// Re-run presolve from the given fixings (NULL: none, the original problem)
// and rebuild the reduced problem on the residual; the constant of variables
// fixed to 1 follows.
int or_fix_variables(void* h, const int8_t* fix) {
  Space& S = *static_cast<Space*>(h);
  const int st = presolve(S, fix);
  if (st != OK) return st;
  if (S.has_cost) {
    S.offset = 0.0;
    for (int64_t p = 0; p < S.nP; ++p)
      if (S.state[p] == 1) S.offset += S.cost[p];
  }
  return OK;
}

int or_project_feasible(void* h, double* d) {
  project_feasible(*static_cast<Space*>(h), d);
  return OK;
}

int or_subgradient(void* h, const double* lam, double* g) {
  subgradient(*static_cast<Space*>(h), lam, g);
  return OK;
}

int or_lbfgs_direction(int n, int m, const double* Sflat, const double* Yflat, const double* g, double* d) {
  std::vector<std::vector<double>> Sh(m), Yh(m);
  for (int j = 0; j < m; ++j) {
    Sh[j].assign(Sflat + size_t(j) * n, Sflat + size_t(j + 1) * n);
    Yh[j].assign(Yflat + size_t(j) * n, Yflat + size_t(j + 1) * n);
  }
  std::vector<double> gv(g, g + n), dv;
  lbfgs_direction(Sh, Yh, gv, dv);
  std::copy(dv.begin(), dv.end(), d);
  return OK;
}

// FindStepSize on the concave parabola E(gamma) = -(gamma - c)^2 (checks)
double or_find_step_parabola(double c, double gamma, int K, double a_up, double a_down, double dmin,
                             double* E_best) {
  auto E_at = [&](double gm) { return -(gm - c) * (gm - c); };
  StepResult r = find_step(E_at, E_at(0.0), gamma, K, a_up, a_down, dmin);
  if (E_best) *E_best = r.E_best;
  return r.gamma;
}

// L_T at lam = c / deg + phi for given element costs (finite-difference checks)
double or_smoothed_value_phi(void* h, const double* cost, const double* phi, double T) {
  Space& S = *static_cast<Space*>(h);
  const int64_t nnz = int64_t(S.rent_var.size());
  std::vector<double> lam(static_cast<size_t>(nnz));
  double off = 0.0;
  for (int64_t p = 0; p < S.nP; ++p)
    if (S.state[p] == 1) off += cost[p];
  for (size_t i = 0; i < S.free_var.size(); ++i)
    for (int64_t e : S.var_ents[i]) lam[e] = cost[S.free_var[i]] / S.deg[i] + phi[e];
  double save = S.offset;
  S.offset = off;
  double v = sweep(S, lam.data(), T, nullptr, nullptr, nullptr);
  S.offset = save;
  return v;
}

int or_costs_for(void* h, const float* DX, const float* DY, int D, double* cost) {
  Space& S = *static_cast<Space*>(h);
  Space tmp;
  tmp.X = S.X;
  tmp.Y = S.Y;
  tmp.pv = S.pv;
  tmp.nP = S.nP;
  tmp.state = S.state;
  int st = compute_costs(tmp, DX, DY, D);
  if (st == OK) std::copy(tmp.cost.begin(), tmp.cost.end(), cost);
  return st;
}

}  // extern "C"
