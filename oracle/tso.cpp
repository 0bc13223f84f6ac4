/*
 * tso.cpp -- CPU oracle for scalar-field topological simplification.
 *
 * TEST INFRASTRUCTURE ONLY (see tso.h).  Plain single-threaded C++17,
 * written for readability, not speed.  Every step names the passage of
 * Kissi et al., "A Practical Solver for Scalar Data Topological
 * Simplification" (arXiv 2407.12399) that it follows.
 *
 * Build:  g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared tso.cpp -o liboracle.so
 * (-ffp-contract=off: the gradient step is specified in plain FP32 with no
 * fused multiply-add, so that its rounding is reproducible.)
 */
#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif
#include "tso.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

/* ------------------------------------------------------------------------ */
/* Grid and Kuhn (Freudenthal) cells -- Sec. 2.1                              */
/* ------------------------------------------------------------------------ */

struct Grid {
  int64_t L[3];
  int64_t n;
  bool valid;
  explicit Grid(const int64_t d[3]) {
    valid = d && d[0] >= 2 && d[1] >= 2 && d[2] >= 2;
    for (int i = 0; i < 3; ++i) L[i] = d ? d[i] : 0;
    n = valid ? L[0] * L[1] * L[2] : 0;
    if (valid && n > (int64_t(1) << 27)) valid = false; /* 12n must fit int32 ids */
  }
  void xyz(int64_t v, int64_t c[3]) const {
    c[0] = v % L[0];
    c[1] = (v / L[0]) % L[1];
    c[2] = v / (L[0] * L[1]);
  }
  bool inside(const int64_t c[3]) const {
    return c[0] >= 0 && c[0] < L[0] && c[1] >= 0 && c[1] < L[1] && c[2] >= 0 &&
           c[2] < L[2];
  }
  int64_t vid(const int64_t c[3]) const { return c[0] + L[0] * (c[1] + L[1] * c[2]); }
};

/* Unit-cube corner for a 3-bit mask: bit0 = x, bit1 = y, bit2 = z. */
void corner(int m, int64_t o[3]) {
  o[0] = m & 1;
  o[1] = (m >> 1) & 1;
  o[2] = (m >> 2) & 1;
}

/* Canonical cell types: the Kuhn chain of corner masks of each type (the id
 * convention of tso.h). */
const int kVertChain[1][1] = {{0}};
const int kEdgeChain[7][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}, {0, 6}, {0, 7}};
const int kTriChain[12][3] = {{0, 1, 3}, {0, 2, 3}, {0, 1, 5}, {0, 4, 5},
                              {0, 2, 6}, {0, 4, 6}, {0, 1, 7}, {0, 2, 7},
                              {0, 3, 7}, {0, 4, 7}, {0, 5, 7}, {0, 6, 7}};
const int kTetChain[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7},
                             {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
const int kNumTypes[4] = {1, 7, 12, 6};

int chain_mask(int dim, int type, int k) {
  switch (dim) {
    case 0: return kVertChain[type][k];
    case 1: return kEdgeChain[type][k];
    case 2: return kTriChain[type][k];
    default: return kTetChain[type][k];
  }
}

struct Cell {
  int dim = -1;
  int64_t id = -1;
  int64_t v[4] = {-1, -1, -1, -1}; /* vertices, ascending id (chain order) */
};

bool make_cell(const Grid& g, int dim, int64_t id, Cell* c) {
  const int64_t K = kNumTypes[dim];
  if (id < 0) return false;
  const int64_t u = id / K;
  const int t = int(id % K);
  if (u >= g.n) return false;
  int64_t uc[3], o[3], p[3];
  g.xyz(u, uc);
  for (int k = 0; k <= dim; ++k) {
    corner(chain_mask(dim, t, k), o);
    for (int a = 0; a < 3; ++a) p[a] = uc[a] + o[a];
    if (!g.inside(p)) return false;
    c->v[k] = g.vid(p);
  }
  for (int k = dim + 1; k < 4; ++k) c->v[k] = -1;
  c->dim = dim;
  c->id = id;
  return true;
}

/* Canonical id of the cell with the given (ascending) vertices, -1 if the
 * vertices are not a Kuhn chain. */
int64_t id_from_vertices(const Grid& g, int dim, const int64_t* vs) {
  int64_t u[3], p[3];
  g.xyz(vs[0], u);
  int masks[4] = {0, 0, 0, 0};
  for (int k = 1; k <= dim; ++k) {
    g.xyz(vs[k], p);
    int m = 0;
    for (int a = 0; a < 3; ++a) {
      const int64_t d = p[a] - u[a];
      if (d != 0 && d != 1) return -1;
      m |= int(d) << a;
    }
    masks[k] = m;
  }
  for (int t = 0; t < kNumTypes[dim]; ++t) {
    bool same = true;
    for (int k = 0; k <= dim; ++k) same = same && chain_mask(dim, t, k) == masks[k];
    if (same) return kNumTypes[dim] * vs[0] + t;
  }
  return -1;
}

/* All cells of dimension >= 1 that contain vertex x (the star of x).  Each
 * cell is found from its unique anchor (its lowest vertex). */
void star_cells(const Grid& g, int64_t x, std::vector<Cell>* out) {
  out->clear();
  int64_t xc[3], o[3], uc[3];
  g.xyz(x, xc);
  for (int m = 0; m < 8; ++m) {
    corner(m, o);
    for (int a = 0; a < 3; ++a) uc[a] = xc[a] - o[a];
    if (!g.inside(uc)) continue;
    const int64_t u = g.vid(uc);
    for (int dim = 1; dim <= 3; ++dim)
      for (int t = 0; t < kNumTypes[dim]; ++t) {
        bool has = false;
        for (int k = 0; k <= dim; ++k) has = has || chain_mask(dim, t, k) == m;
        if (!has) continue;
        Cell c;
        if (make_cell(g, dim, kNumTypes[dim] * u + t, &c)) out->push_back(c);
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Vertex order and lexicographic keys -- Sec. 2.1, Sec. 2.2                  */
/* ------------------------------------------------------------------------ */

/* Ranks of the cell's vertices sorted decreasingly, padded with -1 so that a
 * proper prefix compares lower (a face precedes its cofaces). */
typedef std::array<int64_t, 4> Key;

Key cell_key(const Cell& c, const int32_t* rank) {
  Key k = {-1, -1, -1, -1};
  for (int i = 0; i <= c.dim; ++i) k[i] = rank[c.v[i]];
  std::sort(k.begin(), k.begin() + c.dim + 1, std::greater<int64_t>());
  return k;
}

int64_t highest_vertex(const Cell& c, const int32_t* rank) {
  int64_t best = c.v[0];
  for (int i = 1; i <= c.dim; ++i)
    if (rank[c.v[i]] > rank[best]) best = c.v[i];
  return best;
}

/* -0.0 is the same value as +0.0 in the vertex order. */
float canon(float x) { return x == 0.0f ? 0.0f : x; }

void vertex_order(const float* f, int64_t n, std::vector<int32_t>* order,
                  std::vector<int32_t>* rank) {
  order->resize(n);
  rank->resize(n);
  for (int64_t i = 0; i < n; ++i) (*order)[i] = int32_t(i);
  auto before = [&](int32_t a, int32_t b) {
    const float fa = canon(f[a]), fb = canon(f[b]);
    if (fa != fb) return fa < fb;
    return a < b;
  };
#ifdef _OPENMP
  /* the multi-core timing build only: a parallel sort under the same total
     order gives the same permutation */
  __gnu_parallel::sort(order->begin(), order->end(), before);
#else
  std::sort(order->begin(), order->end(), before);
#endif
  for (int64_t i = 0; i < n; ++i) (*rank)[(*order)[i]] = int32_t(i);
}

bool all_finite(const float* f, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) return false;
  return true;
}

/* ------------------------------------------------------------------------ */
/* Discrete gradient by lower stars -- Sec. 4.2 (Robins et al.'s algorithm)   */
/* ------------------------------------------------------------------------ */

struct LowerStar {
  int64_t x = -1;
  std::vector<Cell> cells; /* L(x) without x itself (dims 1..3) */
  std::vector<Key> keys;
  std::vector<std::vector<int>> facets;   /* facets in L(x) (those containing x) */
  std::vector<std::vector<int>> cofacets; /* cofacets in L(x) */
};

void build_lower_star(const Grid& g, const int32_t* rank, int64_t x,
                      std::vector<Cell>* scratch, LowerStar* ls) {
  ls->x = x;
  ls->cells.clear();
  ls->keys.clear();
  star_cells(g, x, scratch);
  for (const Cell& c : *scratch) {
    bool lower = true;
    for (int k = 0; k <= c.dim; ++k)
      if (c.v[k] != x && rank[c.v[k]] > rank[x]) lower = false;
    if (lower) {
      ls->cells.push_back(c);
      ls->keys.push_back(cell_key(c, rank));
    }
  }
  const size_t m = ls->cells.size();
  ls->facets.assign(m, {});
  ls->cofacets.assign(m, {});
  for (size_t i = 0; i < m; ++i) {
    const Cell& c = ls->cells[i];
    if (c.dim < 2) continue;
    for (int drop = 0; drop <= c.dim; ++drop) {
      if (c.v[drop] == x) continue;
      int64_t vs[3];
      int k = 0;
      for (int j = 0; j <= c.dim; ++j)
        if (j != drop) vs[k++] = c.v[j];
      const int64_t fid = id_from_vertices(g, c.dim - 1, vs);
      for (size_t j = 0; j < m; ++j)
        if (ls->cells[j].dim == c.dim - 1 && ls->cells[j].id == fid) {
          ls->facets[i].push_back(int(j));
          ls->cofacets[j].push_back(int(i));
        }
    }
  }
}

/* Result of the lower-star pairing of one vertex.  Index -1 denotes x. */
struct LSResult {
  std::vector<std::pair<int, int>> pairs; /* (face, coface) */
  std::vector<int> critical;
};

/* The lower-star algorithm: pair x with its lowest edge, then alternately
 * (a) pair the lowest cell having exactly one unclassified facet with that
 *     facet (queue "one"), and
 * (b) when no such cell is left, declare the lowest unclassified cell of
 *     queue "zero" critical,
 * where priorities are lexicographic keys and a facet is "unclassified" when
 * it is neither paired nor critical.  Cells found already classified when
 * popped are skipped. */
void process_lower_star(const LowerStar& ls, LSResult* res) {
  res->pairs.clear();
  res->critical.clear();
  const int m = int(ls.cells.size());
  int first_edge = -1;
  for (int i = 0; i < m; ++i)
    if (ls.cells[i].dim == 1 &&
        (first_edge < 0 || ls.keys[i] < ls.keys[first_edge]))
      first_edge = i;
  if (first_edge < 0) { /* L(x) = {x}: x is a minimum */
    res->critical.push_back(-1);
    return;
  }
  std::vector<char> classified(m, 0);
  auto unclassified_facets = [&](int a, int* last) {
    int cnt = 0;
    for (int f : ls.facets[a])
      if (!classified[f]) {
        ++cnt;
        *last = f;
      }
    return cnt;
  };
  typedef std::pair<Key, int> Item;
  std::set<Item> pq_zero, pq_one;
  auto push_one_cofacets = [&](int c) {
    for (int b : ls.cofacets[c]) {
      int dummy;
      if (unclassified_facets(b, &dummy) == 1) pq_one.insert(Item(ls.keys[b], b));
    }
  };

  res->pairs.push_back({-1, first_edge});
  classified[first_edge] = 1;
  for (int i = 0; i < m; ++i)
    if (ls.cells[i].dim == 1 && i != first_edge) pq_zero.insert(Item(ls.keys[i], i));
  push_one_cofacets(first_edge);

  while (!pq_one.empty() || !pq_zero.empty()) {
    while (!pq_one.empty()) {
      const int a = pq_one.begin()->second;
      pq_one.erase(pq_one.begin());
      if (classified[a]) continue;
      int tau = -1;
      if (unclassified_facets(a, &tau) == 0) {
        pq_zero.insert(Item(ls.keys[a], a));
      } else {
        res->pairs.push_back({tau, a});
        classified[tau] = 1;
        classified[a] = 1;
        push_one_cofacets(a);
        push_one_cofacets(tau);
      }
    }
    if (!pq_zero.empty()) {
      const int c = pq_zero.begin()->second;
      pq_zero.erase(pq_zero.begin());
      if (classified[c]) continue;
      classified[c] = 1;
      res->critical.push_back(c);
      push_one_cofacets(c);
    }
  }
}

/* Whole-field gradient as partner arrays over canonical ids. */
struct Gradient {
  std::vector<int64_t> vup, eup, tup;      /* coface partner, -1 none, -2 invalid */
  std::vector<int64_t> edown, tdown, qdown; /* face partner, -1 none, -2 invalid */
};

void compute_gradient(const Grid& g, const int32_t* rank, Gradient* G) {
  const int64_t n = g.n;
  G->vup.assign(n, -1);
  G->eup.assign(7 * n, -2);
  G->tup.assign(12 * n, -2);
  G->edown.assign(7 * n, -2);
  G->tdown.assign(12 * n, -2);
  G->qdown.assign(6 * n, -2);
  /* The multi-core timing build (-fopenmp) splits these loops over threads;
     every cell lies in the lower star of exactly one vertex (its highest),
     so the writes of different vertices never meet and the result is the
     single-threaded one.  The checker is built without OpenMP. */
#pragma omp parallel
  {
    Cell c;
#pragma omp for schedule(static)
    for (int64_t id = 0; id < 7 * n; ++id)
      if (make_cell(g, 1, id, &c)) G->eup[id] = G->edown[id] = -1;
#pragma omp for schedule(static)
    for (int64_t id = 0; id < 12 * n; ++id)
      if (make_cell(g, 2, id, &c)) G->tup[id] = G->tdown[id] = -1;
#pragma omp for schedule(static)
    for (int64_t id = 0; id < 6 * n; ++id)
      if (make_cell(g, 3, id, &c)) G->qdown[id] = -1;

    std::vector<Cell> scratch;
    LowerStar ls;
    LSResult res;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t x = 0; x < n; ++x) {
      build_lower_star(g, rank, x, &scratch, &ls);
      process_lower_star(ls, &res);
      for (const auto& pr : res.pairs) {
        const Cell& hi = ls.cells[pr.second];
        if (pr.first < 0) {
          G->vup[x] = hi.id;
          G->edown[hi.id] = x;
          continue;
        }
        const Cell& lo = ls.cells[pr.first];
        if (lo.dim == 1) {
          G->eup[lo.id] = hi.id;
          G->tdown[hi.id] = lo.id;
        } else {
          G->tup[lo.id] = hi.id;
          G->qdown[hi.id] = lo.id;
        }
      }
    }
  }
}

bool is_critical(const Gradient& G, int dim, int64_t id) {
  switch (dim) {
    case 0: return G.vup[id] == -1;
    case 1: return G.eup[id] == -1 && G.edown[id] == -1;
    case 2: return G.tup[id] == -1 && G.tdown[id] == -1;
    default: return G.qdown[id] == -1;
  }
}

/* Critical cells of each dimension sorted by lexicographic key. */
void critical_cells(const Grid& g, const int32_t* rank, const Gradient& G,
                    std::vector<Cell> crit[4]) {
  Cell c;
  for (int dim = 0; dim < 4; ++dim) {
    crit[dim].clear();
    const int64_t N = kNumTypes[dim] * g.n;
    for (int64_t id = 0; id < N; ++id)
      if (make_cell(g, dim, id, &c) && is_critical(G, dim, id)) crit[dim].push_back(c);
    std::sort(crit[dim].begin(), crit[dim].end(), [&](const Cell& a, const Cell& b) {
      return cell_key(a, rank) < cell_key(b, rank);
    });
  }
}

/* ------------------------------------------------------------------------ */
/* Persistence pairs                                                          */
/* ------------------------------------------------------------------------ */

struct RawPair {
  int dim;
  int64_t birth, death; /* canonical ids; death -1 for the essential class */
};

/* Tetrahedra containing a triangle (1 on the box boundary, else 2). */
void triangle_cofacets(const Grid& g, const Cell& t, std::vector<Cell>* scratch,
                       int64_t out[2], int* cnt) {
  *cnt = 0;
  star_cells(g, t.v[0], scratch);
  for (const Cell& c : *scratch) {
    if (c.dim != 3) continue;
    int hit = 0;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) hit += c.v[k] == t.v[i];
    if (hit == 3) out[(*cnt)++] = c.id;
  }
}

struct UnionFind {
  std::vector<int64_t> parent;
  explicit UnionFind(int64_t n) : parent(n) {
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
  }
  int64_t find(int64_t a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  }
};

/* Pairing restricted to critical cells (Sec. 4.2, second step):
 *  dim 0: every critical edge, in increasing key order, joins the minima that
 *         the descending gradient paths of its two vertices reach; when the
 *         two components differ, the younger (higher) minimum dies (elder
 *         rule, Sec. 2.2);
 *  dim 2: dually, every critical triangle, in decreasing key order, joins the
 *         maxima (or the outside of the box) that the ascending paths from
 *         its two tetrahedra reach; when they differ the younger (lower)
 *         maximum dies; the outside is older than every maximum;
 *  dim 1: the boundary of each remaining critical triangle, counted mod 2
 *         along gradient paths down to critical edges, is reduced column by
 *         column in increasing order; the highest-key row of a reduced column
 *         is the edge it is paired with. */
void dms_pairs(const Grid& g, const int32_t* rank, const Gradient& G,
               std::vector<RawPair>* out) {
  out->clear();
  std::vector<Cell> crit[4];
  critical_cells(g, rank, G, crit);
  std::vector<Cell> scratch;
  Cell c;

  /* --- dim 0 --- */
  std::vector<int64_t> min_of(g.n, -1);
  auto descend = [&](int64_t v) {
    std::vector<int64_t> path;
    int64_t w = v;
    while (min_of[w] < 0 && G.vup[w] >= 0) {
      path.push_back(w);
      Cell e;
      make_cell(g, 1, G.vup[w], &e);
      w = (e.v[0] == w) ? e.v[1] : e.v[0];
    }
    const int64_t root = min_of[w] >= 0 ? min_of[w] : w;
    min_of[w] = root;
    for (int64_t p : path) min_of[p] = root;
    return root;
  };
  UnionFind uf0(g.n);
  std::vector<char> edge_negative(7 * g.n, 0);
  for (const Cell& e : crit[1]) {
    const int64_t ra = uf0.find(descend(e.v[0]));
    const int64_t rb = uf0.find(descend(e.v[1]));
    if (ra == rb) continue; /* creates a 1-cycle */
    const int64_t younger = rank[ra] > rank[rb] ? ra : rb;
    const int64_t elder = younger == ra ? rb : ra;
    uf0.parent[younger] = elder;
    edge_negative[e.id] = 1;
    out->push_back({0, younger, e.id});
  }
  const int64_t global_min = crit[0].empty() ? 0 : crit[0][0].v[0];
  out->push_back({0, global_min, -1});

  /* --- dim 2 --- */
  const int64_t OUTSIDE = 6 * g.n;
  std::vector<int64_t> max_of(6 * g.n, -1);
  std::vector<Key> tet_key(6 * g.n);
  auto ascend = [&](int64_t T) {
    std::vector<int64_t> path;
    int64_t w = T;
    while (w != OUTSIDE && max_of[w] < 0 && G.qdown[w] >= 0) {
      path.push_back(w);
      Cell t;
      make_cell(g, 2, G.qdown[w], &t);
      int64_t cof[2];
      int cnt;
      triangle_cofacets(g, t, &scratch, cof, &cnt);
      int64_t next = OUTSIDE;
      for (int i = 0; i < cnt; ++i)
        if (cof[i] != w) next = cof[i];
      w = next;
    }
    const int64_t root = (w == OUTSIDE) ? OUTSIDE : (max_of[w] >= 0 ? max_of[w] : w);
    if (w != OUTSIDE) max_of[w] = root;
    for (int64_t p : path) max_of[p] = root;
    return root;
  };
  for (const Cell& T : crit[3]) tet_key[T.id] = cell_key(T, rank);
  UnionFind uf2(6 * g.n + 1);
  auto elder_of = [&](int64_t a, int64_t b) {
    if (a == OUTSIDE || b == OUTSIDE) return OUTSIDE;
    return tet_key[a] > tet_key[b] ? a : b;
  };
  std::vector<char> tri_positive(12 * g.n, 0);
  for (auto it = crit[2].rbegin(); it != crit[2].rend(); ++it) {
    const Cell& t = *it;
    int64_t cof[2];
    int cnt;
    triangle_cofacets(g, t, &scratch, cof, &cnt);
    const int64_t r1 = uf2.find(ascend(cof[0]));
    const int64_t r2 = uf2.find(cnt == 2 ? ascend(cof[1]) : OUTSIDE);
    if (r1 == r2) continue; /* kills a 1-cycle */
    const int64_t elder = elder_of(r1, r2);
    const int64_t younger = elder == r1 ? r2 : r1;
    uf2.parent[younger] = elder;
    tri_positive[t.id] = 1;
    out->push_back({2, t.id, younger});
  }

  /* --- dim 1 --- */
  auto edge_key = [&](int64_t id) {
    make_cell(g, 1, id, &c);
    return cell_key(c, rank);
  };
  std::map<Key, int64_t> owner_of_row; /* pivot row -> column index */
  std::vector<std::vector<std::pair<Key, int64_t>>> reduced;
  for (const Cell& t : crit[2]) {
    if (tri_positive[t.id]) continue; /* clearing: positive triangles */
    /* Morse boundary: expand non-critical edges along the gradient, mod 2. */
    std::map<Key, int64_t> work, bnd;
    auto toggle = [](std::map<Key, int64_t>& s, const Key& k, int64_t id) {
      auto f = s.find(k);
      if (f != s.end()) s.erase(f);
      else s.emplace(k, id);
    };
    for (int drop = 0; drop < 3; ++drop) {
      int64_t vs[2];
      int k = 0;
      for (int j = 0; j < 3; ++j)
        if (j != drop) vs[k++] = t.v[j];
      const int64_t e = id_from_vertices(g, 1, vs);
      toggle(work, edge_key(e), e);
    }
    while (!work.empty()) {
      auto top = std::prev(work.end());
      const int64_t e = top->second;
      const Key ek = top->first;
      work.erase(top);
      if (is_critical(G, 1, e)) {
        toggle(bnd, ek, e);
      } else if (G.eup[e] >= 0) {
        Cell tri, ec;
        make_cell(g, 2, G.eup[e], &tri);
        make_cell(g, 1, e, &ec);
        for (int drop = 0; drop < 3; ++drop) {
          int64_t vs[2];
          int k = 0;
          for (int j = 0; j < 3; ++j)
            if (j != drop) vs[k++] = tri.v[j];
          const int64_t f = id_from_vertices(g, 1, vs);
          if (f != e) toggle(work, edge_key(f), f);
        }
      } /* else: paired with a vertex, the path ends without contribution */
    }
    std::vector<std::pair<Key, int64_t>> col;
    for (auto it = bnd.rbegin(); it != bnd.rend(); ++it)
      if (!edge_negative[it->second]) col.push_back(*it); /* descending */
    while (!col.empty()) {
      auto own = owner_of_row.find(col.front().first);
      if (own == owner_of_row.end()) break;
      const auto& other = reduced[own->second];
      std::vector<std::pair<Key, int64_t>> sum;
      std::set_symmetric_difference(
          col.begin(), col.end(), other.begin(), other.end(), std::back_inserter(sum),
          [](const std::pair<Key, int64_t>& a, const std::pair<Key, int64_t>& b) {
            return a.first > b.first;
          });
      col.swap(sum);
    }
    if (col.empty()) continue; /* cannot happen for a negative triangle */
    owner_of_row[col.front().first] = int64_t(reduced.size());
    out->push_back({1, col.front().second, t.id});
    reduced.push_back(col);
  }
}

/* Definition: standard Z2 reduction of the boundary matrix of the whole
 * lexicographic filtration (Sec. 2.2), with clearing. */
void full_reduction_pairs(const Grid& g, const int32_t* rank, std::vector<RawPair>* out) {
  out->clear();
  std::vector<Cell> cells;
  Cell c;
  for (int dim = 0; dim < 4; ++dim)
    for (int64_t id = 0; id < kNumTypes[dim] * g.n; ++id)
      if (make_cell(g, dim, id, &c)) cells.push_back(c);
  const int64_t N = int64_t(cells.size());
  std::vector<Key> keys(N);
  for (int64_t i = 0; i < N; ++i) keys[i] = cell_key(cells[i], rank);
  std::vector<int64_t> ord(N);
  for (int64_t i = 0; i < N; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  std::vector<int64_t> pos_of[4];
  for (int dim = 0; dim < 4; ++dim) pos_of[dim].assign(kNumTypes[dim] * g.n, -1);
  for (int64_t p = 0; p < N; ++p) pos_of[cells[ord[p]].dim][cells[ord[p]].id] = p;

  std::vector<std::vector<int64_t>> col(N); /* ascending positions */
  for (int64_t p = 0; p < N; ++p) {
    const Cell& s = cells[ord[p]];
    if (s.dim == 0) continue;
    for (int drop = 0; drop <= s.dim; ++drop) {
      int64_t vs[3];
      int k = 0;
      for (int j = 0; j <= s.dim; ++j)
        if (j != drop) vs[k++] = s.v[j];
      col[p].push_back(pos_of[s.dim - 1][id_from_vertices(g, s.dim - 1, vs)]);
    }
    std::sort(col[p].begin(), col[p].end());
  }
  std::vector<int64_t> owner(N, -1);
  std::vector<char> cleared(N, 0), paired(N, 0);
  for (int dim = 3; dim >= 1; --dim) {
    for (int64_t p = 0; p < N; ++p) {
      if (cells[ord[p]].dim != dim || cleared[p]) continue;
      std::vector<int64_t>& cp = col[p];
      while (!cp.empty() && owner[cp.back()] >= 0) {
        std::vector<int64_t> sum;
        const std::vector<int64_t>& o = col[owner[cp.back()]];
        std::set_symmetric_difference(cp.begin(), cp.end(), o.begin(), o.end(),
                                      std::back_inserter(sum));
        cp.swap(sum);
      }
      if (cp.empty()) continue;
      const int64_t low = cp.back();
      owner[low] = p;
      cleared[low] = 1;
      paired[low] = paired[p] = 1;
      out->push_back({cells[ord[low]].dim, cells[ord[low]].id, cells[ord[p]].id});
    }
  }
  for (int64_t p = 0; p < N; ++p)
    if (!paired[p]) out->push_back({cells[ord[p]].dim, cells[ord[p]].id, -1});
}

/* Textbook special cases: Kruskal with the elder rule over all edges (dim 0)
 * and over all triangles of the dual graph with the outside node (dim 2). */
void kruskal_pairs(const Grid& g, const int32_t* rank, std::vector<RawPair>* out) {
  out->clear();
  Cell c;
  std::vector<std::pair<Key, int64_t>> edges, tris;
  for (int64_t id = 0; id < 7 * g.n; ++id)
    if (make_cell(g, 1, id, &c)) edges.push_back({cell_key(c, rank), id});
  std::sort(edges.begin(), edges.end());
  UnionFind uf(g.n);
  for (const auto& e : edges) {
    make_cell(g, 1, e.second, &c);
    const int64_t ra = uf.find(c.v[0]), rb = uf.find(c.v[1]);
    if (ra == rb) continue;
    const int64_t younger = rank[ra] > rank[rb] ? ra : rb;
    uf.parent[younger] = younger == ra ? rb : ra;
    out->push_back({0, younger, e.second});
  }
  int64_t gmin = 0;
  for (int64_t v = 0; v < g.n; ++v)
    if (rank[v] == 0) gmin = v;
  out->push_back({0, gmin, -1});

  for (int64_t id = 0; id < 12 * g.n; ++id)
    if (make_cell(g, 2, id, &c)) tris.push_back({cell_key(c, rank), id});
  std::sort(tris.begin(), tris.end(), std::greater<std::pair<Key, int64_t>>());
  const int64_t OUTSIDE = 6 * g.n;
  std::vector<Key> tkey(6 * g.n);
  for (int64_t id = 0; id < 6 * g.n; ++id)
    if (make_cell(g, 3, id, &c)) tkey[id] = cell_key(c, rank);
  UnionFind uf2(6 * g.n + 1);
  std::vector<Cell> scratch;
  for (const auto& tr : tris) {
    make_cell(g, 2, tr.second, &c);
    int64_t cof[2];
    int cnt;
    triangle_cofacets(g, c, &scratch, cof, &cnt);
    const int64_t r1 = uf2.find(cof[0]);
    const int64_t r2 = uf2.find(cnt == 2 ? cof[1] : OUTSIDE);
    if (r1 == r2) continue;
    int64_t elder;
    if (r1 == OUTSIDE || r2 == OUTSIDE) elder = OUTSIDE;
    else elder = tkey[r1] > tkey[r2] ? r1 : r2;
    const int64_t younger = elder == r1 ? r2 : r1;
    uf2.parent[younger] = elder;
    out->push_back({2, tr.second, younger});
  }
}

void to_records(const Grid& g, const float* f, const int32_t* rank,
                const std::vector<RawPair>& raw, std::vector<tso_pair>* out) {
  out->clear();
  int64_t vmax = 0;
  for (int64_t v = 0; v < g.n; ++v)
    if (rank[v] == g.n - 1) vmax = v;
  Cell b, d;
  for (const RawPair& r : raw) {
    tso_pair p;
    p.dim = r.dim;
    p.essential = r.death < 0;
    p.birth_cell = r.birth;
    p.death_cell = r.death;
    make_cell(g, r.dim, r.birth, &b);
    p.v_birth = highest_vertex(b, rank);
    if (r.death >= 0) {
      make_cell(g, r.dim + 1, r.death, &d);
      p.v_death = highest_vertex(d, rank);
    } else {
      p.v_death = vmax;
    }
    p.birth = f[p.v_birth];
    p.death = f[p.v_death];
    out->push_back(p);
  }
}

/* Diagram D(f) (Sec. 2.2): non-zero-persistence pairs (v_b != v_d) and the
 * essential class; sorted in diagram order (Sec. 2.4) with ties broken by
 * (rank v_death, dim, birth-cell key). */
void diagram_from_pairs(const Grid& g, const int32_t* rank,
                        const std::vector<tso_pair>& all, std::vector<tso_pair>* D) {
  D->clear();
  for (const tso_pair& p : all)
    if (p.essential || p.v_birth != p.v_death) D->push_back(p);
  Cell c;
  std::vector<std::pair<std::array<int64_t, 7>, size_t>> keyed;
  for (size_t i = 0; i < D->size(); ++i) {
    const tso_pair& p = (*D)[i];
    make_cell(g, p.dim, p.birth_cell, &c);
    const Key bk = cell_key(c, rank);
    keyed.push_back({{rank[p.v_birth], rank[p.v_death], p.dim, bk[0], bk[1], bk[2], bk[3]}, i});
  }
  std::sort(keyed.begin(), keyed.end());
  std::vector<tso_pair> sorted;
  for (const auto& k : keyed) sorted.push_back((*D)[k.second]);
  D->swap(sorted);
}

struct Persistence {
  std::vector<int32_t> order, rank;
  std::vector<tso_pair> pairs;   /* all critical pairs + essential */
  std::vector<tso_pair> diagram; /* D(f) in diagram order */
};

void persistence(const Grid& g, const float* f, Persistence* P) {
  vertex_order(f, g.n, &P->order, &P->rank);
  Gradient G;
  compute_gradient(g, P->rank.data(), &G);
  std::vector<RawPair> raw;
  dms_pairs(g, P->rank.data(), G, &raw);
  to_records(g, f, P->rank.data(), raw, &P->pairs);
  diagram_from_pairs(g, P->rank.data(), P->pairs, &P->diagram);
}

/* ------------------------------------------------------------------------ */
/* Assignment -- Eq. (1) with q = 2, Sec. 4.1                                  */
/* ------------------------------------------------------------------------ */

const double kBig = 1e300;

/* Dense Hungarian algorithm (Kuhn-Munkres) for a square cost matrix
 * a[1..N][1..N], in its O(N^3) shortest-augmenting-path form with row and
 * column potentials (u, v), the column-to-row map p and the path links way:
 * the textbook formulation (Kuhn 1955, Munkres 1957; the potentials version
 * as given, e.g., by Lawler, "Combinatorial Optimization", 1976).  Rows are
 * added one at a time; each addition grows a Dijkstra-like search over
 * columns by reduced cost until it reaches a free column, then flips the
 * path.  Returns col_of_row. */
std::vector<int> hungarian(const std::vector<std::vector<double>>& a) {
  const int N = int(a.size());
  std::vector<double> u(N + 1, 0), v(N + 1, 0), minv(N + 1);
  std::vector<int> p(N + 1, 0), way(N + 1, 0);
  std::vector<char> used(N + 1);
  for (int i = 1; i <= N; ++i) {
    p[0] = i;
    int j0 = 0;
    std::fill(minv.begin(), minv.end(), std::numeric_limits<double>::infinity());
    std::fill(used.begin(), used.end(), 0);
    do {
      used[j0] = 1;
      const int i0 = p[j0];
      double delta = std::numeric_limits<double>::infinity();
      int j1 = 0;
      for (int j = 1; j <= N; ++j)
        if (!used[j]) {
          const double cur = a[i0 - 1][j - 1] - u[i0] - v[j];
          if (cur < minv[j]) {
            minv[j] = cur;
            way[j] = j0;
          }
          if (minv[j] < delta) {
            delta = minv[j];
            j1 = j;
          }
        }
      for (int j = 0; j <= N; ++j)
        if (used[j]) {
          u[p[j]] += delta;
          v[j] -= delta;
        } else {
          minv[j] -= delta;
        }
      j0 = j1;
    } while (p[j0] != 0);
    do {
      const int j1 = way[j0];
      p[j0] = p[j1];
      j0 = j1;
    } while (j0);
  }
  std::vector<int> col_of_row(N, -1);
  for (int j = 1; j <= N; ++j)
    if (p[j] > 0) col_of_row[p[j] - 1] = j - 1;
  return col_of_row;
}

double sq(double a) { return a * a; }
double diag_cost(double b, double d) { return sq(d - b) / 2.0; }
double pair_cost(double pb, double pd, double qb, double qd) {
  return sq(pb - qb) + sq(pd - qd);
}

/* Exact assignment of points to targets or the diagonal (augmented diagrams,
 * Sec. 2.3): rows = points + diagonal copies of targets, columns = targets +
 * diagonal copies of points. */
void assign_dense(const std::vector<double>& pb, const std::vector<double>& pd,
                  const std::vector<double>& qb, const std::vector<double>& qd,
                  std::vector<int>* match, double* total) {
  const int m = int(pb.size()), k = int(qb.size());
  match->assign(m, -1);
  *total = 0;
  if (m + k == 0) return;
  const int N = m + k;
  std::vector<std::vector<double>> C(N, std::vector<double>(N, kBig));
  for (int i = 0; i < m; ++i) {
    const double dp = diag_cost(pb[i], pd[i]);
    for (int j = 0; j < k; ++j) {
      const double c = pair_cost(pb[i], pd[i], qb[j], qd[j]);
      if (c < dp + diag_cost(qb[j], qd[j])) C[i][j] = c;
    }
    C[i][k + i] = dp;
  }
  for (int j = 0; j < k; ++j) {
    C[m + j][j] = diag_cost(qb[j], qd[j]);
    for (int i = 0; i < m; ++i) C[m + j][k + i] = 0.0;
  }
  const std::vector<int> col = hungarian(C);
  for (int i = 0; i < m; ++i) {
    if (col[i] < k) {
      (*match)[i] = col[i];
      *total += C[i][col[i]];
    } else {
      *total += diag_cost(pb[i], pd[i]);
    }
  }
  std::vector<char> taken(k, 0);
  for (int i = 0; i < m; ++i)
    if ((*match)[i] >= 0) taken[(*match)[i]] = 1;
  for (int j = 0; j < k; ++j)
    if (!taken[j]) *total += diag_cost(qb[j], qd[j]);
}

/* ------------------------------------------------------------------------ */
/* Bottleneck distance (stability check)                                      */
/* ------------------------------------------------------------------------ */

/* Augmenting-path bipartite matching (Kuhn's algorithm); small inputs. */
bool augment(int l, const std::vector<std::vector<int>>& adj, std::vector<int>* match_r,
             std::vector<char>* seen) {
  for (int r : adj[l]) {
    if ((*seen)[r]) continue;
    (*seen)[r] = 1;
    if ((*match_r)[r] < 0 || augment((*match_r)[r], adj, match_r, seen)) {
      (*match_r)[r] = l;
      return true;
    }
  }
  return false;
}

bool perfect_matching(int L, int R, const std::vector<std::vector<int>>& adj) {
  std::vector<int> match_r(R, -1);
  for (int l = 0; l < L; ++l) {
    std::vector<char> seen(R, 0);
    if (!augment(l, adj, &match_r, &seen)) return false;
  }
  return true;
}

double bottleneck_group(const std::vector<std::pair<double, double>>& A,
                        const std::vector<std::pair<double, double>>& B) {
  const int m = int(A.size()), k = int(B.size());
  auto dinf = [](const std::pair<double, double>& a, const std::pair<double, double>& b) {
    return std::max(std::fabs(a.first - b.first), std::fabs(a.second - b.second));
  };
  auto ddiag = [](const std::pair<double, double>& a) {
    return std::fabs(a.second - a.first) / 2.0;
  };
  std::vector<double> cand = {0.0};
  for (int i = 0; i < m; ++i) {
    cand.push_back(ddiag(A[i]));
    for (int j = 0; j < k; ++j) cand.push_back(dinf(A[i], B[j]));
  }
  for (int j = 0; j < k; ++j) cand.push_back(ddiag(B[j]));
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  auto feasible = [&](double eps) {
    /* left: A (m) + diagonal copies of B (k); right: B (k) + diagonal copies of A (m) */
    std::vector<std::vector<int>> adj(m + k);
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j < k; ++j)
        if (dinf(A[i], B[j]) <= eps) adj[i].push_back(j);
      if (ddiag(A[i]) <= eps) adj[i].push_back(k + i);
    }
    for (int j = 0; j < k; ++j) {
      if (ddiag(B[j]) <= eps) adj[m + j].push_back(j);
      for (int i = 0; i < m; ++i) adj[m + j].push_back(k + i);
    }
    return perfect_matching(m + k, m + k, adj);
  };
  int lo = 0, hi = int(cand.size()) - 1;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (feasible(cand[mid])) hi = mid;
    else lo = mid + 1;
  }
  return cand[lo];
}

/* ------------------------------------------------------------------------ */
/* Solver -- Alg. 1, Sec. 4.1 (direct step), Sec. 4.3 (still pairs)           */
/* ------------------------------------------------------------------------ */

struct Target {
  int dim, essential;
  int64_t vb0, vd0;
  float b, d; /* coordinates in D(f0) */
};

struct Point {
  int dim, essential;
  int64_t vb, vd;
  float b, d;
};

std::vector<Point> points_of(const std::vector<tso_pair>& D) {
  std::vector<Point> P;
  for (const tso_pair& p : D) P.push_back({p.dim, p.essential, p.v_birth, p.v_death, p.birth, p.death});
  return P;
}

/* Canonical form of an assignment among interchangeable items: points with
 * equal (dim, v_b, v_d) and targets with equal (dim, v_b0, v_d0) have equal
 * coordinates, so the optimum does not tell them apart.  Point classes are
 * visited in diagram order; each class receives its multiset of target
 * classes sorted by smallest member id (diagonal last), and each target class
 * hands out its member ids in increasing order. */
void canonicalize(const std::vector<Point>& P, const std::vector<int>& subset,
                  const std::vector<Target>& T, std::vector<int>* phi) {
  std::map<std::array<int64_t, 3>, std::vector<int>> pclass; /* key -> point ids (diagram order) */
  std::vector<std::array<int64_t, 3>> pclass_order;
  for (int i : subset) {
    const std::array<int64_t, 3> k = {P[i].dim, P[i].vb, P[i].vd};
    auto& v = pclass[k];
    if (v.empty()) pclass_order.push_back(k);
    v.push_back(i);
  }
  std::map<std::array<int64_t, 3>, std::vector<int>> tclass; /* key -> target ids used */
  std::map<int, std::array<int64_t, 3>> tkey_of;
  for (int i : subset)
    if ((*phi)[i] >= 0) {
      const Target& t = T[(*phi)[i]];
      const std::array<int64_t, 3> k = {t.dim, t.vb0, t.vd0};
      tclass[k].push_back((*phi)[i]);
      tkey_of[(*phi)[i]] = k;
    }
  std::map<std::array<int64_t, 3>, size_t> next;
  for (auto& kv : tclass) {
    std::sort(kv.second.begin(), kv.second.end());
    next[kv.first] = 0;
  }
  for (const auto& pk : pclass_order) {
    const std::vector<int>& members = pclass[pk];
    std::vector<std::pair<int64_t, std::array<int64_t, 3>>> got; /* (min id or INF, class) */
    for (int i : members) {
      if ((*phi)[i] < 0) {
        got.push_back({std::numeric_limits<int64_t>::max(), {-1, -1, -1}});
      } else {
        const auto& k = tkey_of[(*phi)[i]];
        got.push_back({tclass[k].front(), k});
      }
    }
    std::sort(got.begin(), got.end());
    for (size_t s = 0; s < members.size(); ++s) {
      if (got[s].second[0] < 0) {
        (*phi)[members[s]] = -1;
      } else {
        const auto& k = got[s].second;
        (*phi)[members[s]] = tclass[k][next[k]++];
      }
    }
  }
}

struct Solver {
  const Grid& g;
  std::vector<Target> T;
  int ess_target = -1;

  explicit Solver(const Grid& grid) : g(grid) {}

  /* Signal selection (Sec. 3) and target diagram D_T = D(f0) minus the
   * non-signal pairs. */
  void build_targets(const std::vector<Point>& P0, const std::vector<tso_pair>& D0,
                     const tso_signal* sig, double range, std::vector<int>* phi0) {
    phi0->assign(P0.size(), -1);
    const double thr = double(sig->threshold_rel) * range;
    for (size_t i = 0; i < P0.size(); ++i) {
      const Point& p = P0[i];
      bool signal;
      if (p.essential) {
        signal = true;
      } else if (sig->mode == 1) {
        signal = false;
        for (int64_t s = 0; s < sig->n_signal; ++s)
          if (sig->signal[s].dim == p.dim && sig->signal[s].birth_cell == D0[i].birth_cell &&
              sig->signal[s].death_cell == D0[i].death_cell)
            signal = true;
      } else {
        const double pers = double(p.d) - double(p.b);
        const bool masked = (sig->nonsignal_dim_mask >> p.dim) & 1u;
        const bool below = pers < thr || (pers == thr && !sig->ties_signal);
        signal = !(masked && below);
      }
      if (signal) {
        if (p.essential) ess_target = int(T.size());
        (*phi0)[i] = int(T.size());
        T.push_back({p.dim, p.essential, p.vb, p.vd, p.b, p.d});
      }
    }
  }

  /* Still pairs (Sec. 4.3): same (dim, v_b, v_d) as a point of the previous
   * diagram; duplicates matched in diagram order.  Still points keep their
   * assignment; the rest is solved exactly per dimension against the targets
   * that no still point holds. */
  void assign(const std::vector<Point>& P, const std::vector<Point>& Pprev,
              const std::vector<int>& phiPrev, std::vector<int>* phi, int64_t* n_still,
              int64_t* n_reduced) {
    phi->assign(P.size(), -1);
    std::map<std::array<int64_t, 3>, std::deque<int>> prev;
    for (size_t i = 0; i < Pprev.size(); ++i)
      prev[{Pprev[i].dim, Pprev[i].vb, Pprev[i].vd}].push_back(int(i));
    std::vector<char> still(P.size(), 0), held(T.size(), 0);
    *n_still = 0;
    for (size_t i = 0; i < P.size(); ++i) {
      auto it = prev.find({P[i].dim, P[i].vb, P[i].vd});
      if (it == prev.end() || it->second.empty()) continue;
      const int j = it->second.front();
      it->second.pop_front();
      still[i] = 1;
      ++*n_still;
      (*phi)[i] = phiPrev[j];
      if ((*phi)[i] >= 0) held[(*phi)[i]] = 1;
    }
    std::vector<int> reduced_pts;
    for (size_t i = 0; i < P.size(); ++i) {
      if (P[i].essential) {
        if (!still[i]) (*phi)[i] = ess_target;
        continue;
      }
      if (!still[i]) reduced_pts.push_back(int(i));
    }
    *n_reduced = int64_t(reduced_pts.size());
    for (int dim = 0; dim < 3; ++dim) {
      std::vector<int> pi, tj;
      std::vector<double> pb, pd, qb, qd;
      for (int i : reduced_pts)
        if (P[i].dim == dim) {
          pi.push_back(i);
          pb.push_back(P[i].b);
          pd.push_back(P[i].d);
        }
      for (size_t j = 0; j < T.size(); ++j)
        if (!held[j] && !T[j].essential && T[j].dim == dim) {
          tj.push_back(int(j));
          qb.push_back(T[j].b);
          qd.push_back(T[j].d);
        }
      std::vector<int> match;
      double total;
      assign_dense(pb, pd, qb, qd, &match, &total);
      for (size_t s = 0; s < pi.size(); ++s) (*phi)[pi[s]] = match[s] >= 0 ? tj[match[s]] : -1;
    }
    canonicalize(P, reduced_pts, T, phi);
  }

  /* L(v_f) = sum over diagram points of the squared distance to the assigned
   * target or diagonal projection (Sec. 4.1). */
  double loss(const std::vector<Point>& P, const std::vector<int>& phi) const {
    double L = 0;
    for (size_t i = 0; i < P.size(); ++i) {
      if (phi[i] >= 0)
        L += pair_cost(P[i].b, P[i].d, T[phi[i]].b, T[phi[i]].d);
      else
        L += diag_cost(P[i].b, P[i].d);
    }
    return L;
  }

  double unmatched_target_cost(const std::vector<int>& phi) const {
    std::vector<char> used(T.size(), 0);
    for (int t : phi)
      if (t >= 0) used[t] = 1;
    double s = 0;
    for (size_t j = 0; j < T.size(); ++j)
      if (!used[j]) s += diag_cost(T[j].b, T[j].d);
    return s;
  }

  double max_diag_pers(const std::vector<Point>& P, const std::vector<int>& phi) const {
    double m = 0;
    for (size_t i = 0; i < P.size(); ++i)
      if (phi[i] < 0) m = std::max(m, double(P[i].d) - double(P[i].b));
    return m;
  }

  /* Direct gradient step (Sec. 4.1): for every point, in diagram order,
   * g_b = 2 (x[v_b] - t_b) and g_d = 2 (x[v_d] - t_d) in FP32; per vertex the
   * birth and death gradients are summed in that order; then
   * x <- x - (alpha_b * B + alpha_d * D).  Diagonal targets are the diagonal
   * projection ((b+d)/2, (b+d)/2) of the current point. */
  void step(std::vector<float>* x, const std::vector<Point>& P, const std::vector<int>& phi,
            float alpha_b, float alpha_d) const {
    std::vector<float> B(x->size(), 0.0f), Dg(x->size(), 0.0f);
    std::vector<char> touched(x->size(), 0);
    for (size_t i = 0; i < P.size(); ++i) {
      float tb, td;
      if (phi[i] >= 0) {
        tb = T[phi[i]].b;
        td = T[phi[i]].d;
      } else {
        const float mid = (P[i].b + P[i].d) * 0.5f;
        tb = td = mid;
      }
      const float gb = 2.0f * ((*x)[P[i].vb] - tb);
      const float gd = 2.0f * ((*x)[P[i].vd] - td);
      B[P[i].vb] = B[P[i].vb] + gb;
      Dg[P[i].vd] = Dg[P[i].vd] + gd;
      touched[P[i].vb] = touched[P[i].vd] = 1;
    }
    for (size_t v = 0; v < x->size(); ++v)
      if (touched[v]) {
        const float db = alpha_b * B[v];
        const float dd = alpha_d * Dg[v];
        const float s = db + dd;
        (*x)[v] = canon((*x)[v] - s);
      }
  }
};

}  // namespace

/* ======================================================================== */
/* C ABI                                                                     */
/* ======================================================================== */

extern "C" {

int tso_order(const float* f, int64_t n, int32_t* order, int32_t* rank) {
  if (!f || !order || !rank || n <= 0 || n > (int64_t(1) << 31) - 1) return -1;
  if (!all_finite(f, n)) return -2;
  std::vector<int32_t> o, r;
  vertex_order(f, n, &o, &r);
  std::memcpy(order, o.data(), sizeof(int32_t) * n);
  std::memcpy(rank, r.data(), sizeof(int32_t) * n);
  return 0;
}

int tso_gradient(const float* f, const int64_t dims[3], int32_t* vup, int32_t* eup,
                 int32_t* tup) {
  Grid g(dims);
  if (!g.valid || !f || !vup || !eup || !tup) return -1;
  if (!all_finite(f, g.n)) return -2;
  std::vector<int32_t> order, rank;
  vertex_order(f, g.n, &order, &rank);
  Gradient G;
  compute_gradient(g, rank.data(), &G);
  for (int64_t i = 0; i < g.n; ++i) vup[i] = int32_t(G.vup[i]);
  for (int64_t i = 0; i < 7 * g.n; ++i) eup[i] = int32_t(G.eup[i]);
  for (int64_t i = 0; i < 12 * g.n; ++i) tup[i] = int32_t(G.tup[i]);
  return 0;
}

int tso_gradient_at(const int32_t* rank, const int64_t dims[3], int64_t v,
                    int32_t* pair_dim, int64_t* pair_face, int64_t* pair_coface,
                    int32_t* n_pairs, int32_t* crit_dim, int64_t* crit_id, int32_t* n_crit) {
  Grid g(dims);
  if (!g.valid || !rank || v < 0 || v >= g.n) return -1;
  std::vector<Cell> scratch;
  LowerStar ls;
  LSResult res;
  build_lower_star(g, rank, v, &scratch, &ls);
  process_lower_star(ls, &res);
  std::vector<std::array<int64_t, 3>> prs;
  for (const auto& pr : res.pairs) {
    const Cell& hi = ls.cells[pr.second];
    const int64_t lo_id = pr.first < 0 ? v : ls.cells[pr.first].id;
    prs.push_back({hi.dim - 1, lo_id, hi.id});
  }
  std::sort(prs.begin(), prs.end());
  std::vector<std::pair<int64_t, int64_t>> crs;
  for (int c : res.critical) {
    if (c < 0) crs.push_back({0, v});
    else crs.push_back({ls.cells[c].dim, ls.cells[c].id});
  }
  std::sort(crs.begin(), crs.end());
  *n_pairs = int32_t(prs.size());
  for (size_t i = 0; i < prs.size(); ++i) {
    pair_dim[i] = int32_t(prs[i][0]);
    pair_face[i] = prs[i][1];
    pair_coface[i] = prs[i][2];
  }
  *n_crit = int32_t(crs.size());
  for (size_t i = 0; i < crs.size(); ++i) {
    crit_dim[i] = int32_t(crs[i].first);
    crit_id[i] = crs[i].second;
  }
  return 0;
}

int tso_critical(const float* f, const int64_t dims[3], int32_t* out_dim, int64_t* out_id,
                 int64_t capacity, int64_t* n_out) {
  Grid g(dims);
  if (!g.valid || !f || !n_out) return -1;
  if (!all_finite(f, g.n)) return -2;
  std::vector<int32_t> order, rank;
  vertex_order(f, g.n, &order, &rank);
  Gradient G;
  compute_gradient(g, rank.data(), &G);
  std::vector<Cell> crit[4];
  critical_cells(g, rank.data(), G, crit);
  int64_t total = 0;
  for (int d = 0; d < 4; ++d) total += int64_t(crit[d].size());
  *n_out = total;
  if (total > capacity || !out_dim || !out_id) return total > capacity ? -5 : -1;
  int64_t k = 0;
  for (int d = 0; d < 4; ++d)
    for (const Cell& c : crit[d]) {
      out_dim[k] = d;
      out_id[k++] = c.id;
    }
  return 0;
}

int tso_pairs(const float* f, const int64_t dims[3], int32_t method, tso_pair* out,
              int64_t capacity, int64_t* n_out) {
  Grid g(dims);
  if (!g.valid || !f || !n_out || method < 0 || method > 2) return -1;
  if (!all_finite(f, g.n)) return -2;
  std::vector<int32_t> order, rank;
  vertex_order(f, g.n, &order, &rank);
  std::vector<RawPair> raw;
  if (method == 0) {
    Gradient G;
    compute_gradient(g, rank.data(), &G);
    dms_pairs(g, rank.data(), G, &raw);
  } else if (method == 1) {
    full_reduction_pairs(g, rank.data(), &raw);
  } else {
    kruskal_pairs(g, rank.data(), &raw);
  }
  std::vector<tso_pair> recs;
  to_records(g, f, rank.data(), raw, &recs);
  std::sort(recs.begin(), recs.end(), [](const tso_pair& a, const tso_pair& b) {
    if (a.dim != b.dim) return a.dim < b.dim;
    if (a.birth_cell != b.birth_cell) return a.birth_cell < b.birth_cell;
    return a.death_cell < b.death_cell;
  });
  *n_out = int64_t(recs.size());
  if (int64_t(recs.size()) > capacity) return -5;
  if (!out && !recs.empty()) return -1;
  std::copy(recs.begin(), recs.end(), out);
  return 0;
}

int tso_diagram(const float* f, const int64_t dims[3], tso_pair* out, int64_t capacity,
                int64_t* n_out) {
  Grid g(dims);
  if (!g.valid || !f || !n_out) return -1;
  if (!all_finite(f, g.n)) return -2;
  Persistence P;
  persistence(g, f, &P);
  *n_out = int64_t(P.diagram.size());
  if (int64_t(P.diagram.size()) > capacity) return -5;
  if (!out) return -1;
  std::copy(P.diagram.begin(), P.diagram.end(), out);
  return 0;
}

int tso_assign(int64_t n_pts, const double* pb, const double* pd, int64_t n_tgt,
               const double* qb, const double* qd, int32_t* match, double* cost) {
  if (n_pts < 0 || n_tgt < 0 || !match || !cost) return -1;
  std::vector<double> PB(pb, pb + n_pts), PD(pd, pd + n_pts), QB(qb, qb + n_tgt),
      QD(qd, qd + n_tgt);
  std::vector<int> m;
  assign_dense(PB, PD, QB, QD, &m, cost);
  for (int64_t i = 0; i < n_pts; ++i) match[i] = m[i];
  return 0;
}

int tso_assign_step(const tso_pair* prev, int64_t n_prev, const int32_t* phi_prev,
                    const tso_pair* cur, int64_t n_cur, const tso_pair* targets,
                    int64_t n_tgt, int32_t* phi_out, int64_t* n_still, int64_t* n_reduced) {
  if (n_prev < 0 || n_cur < 0 || n_tgt < 0 || !phi_out || !n_still || !n_reduced) return -1;
  if ((n_prev > 0 && (!prev || !phi_prev)) || (n_cur > 0 && !cur) || (n_tgt > 0 && !targets))
    return -1;
  const int64_t dims[3] = {2, 2, 2};
  Grid g(dims);
  Solver S(g);
  for (int64_t j = 0; j < n_tgt; ++j) {
    const tso_pair& t = targets[j];
    if (t.essential) {
      if (S.ess_target >= 0) return -1;
      S.ess_target = int(j);
    }
    S.T.push_back({t.dim, t.essential, t.v_birth, t.v_death, t.birth, t.death});
  }
  std::vector<tso_pair> A(prev, prev + n_prev), B(cur, cur + n_cur);
  const std::vector<Point> Pp = points_of(A), Pc = points_of(B);
  std::vector<int> phip(n_prev);
  for (int64_t i = 0; i < n_prev; ++i) {
    if (phi_prev[i] < -1 || phi_prev[i] >= n_tgt) return -1;
    phip[i] = phi_prev[i];
  }
  for (const Point& p : Pc)
    if (p.essential && S.ess_target < 0) return -1;
  std::vector<int> phi;
  S.assign(Pc, Pp, phip, &phi, n_still, n_reduced);
  for (int64_t i = 0; i < n_cur; ++i) phi_out[i] = phi[i];
  return 0;
}

int tso_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int tso_bottleneck(const tso_pair* a, int64_t na, const tso_pair* b, int64_t nb,
                   double* out) {
  if (!out || na < 0 || nb < 0) return -1;
  double worst = 0;
  for (int group = 0; group < 4; ++group) { /* dims 0..2 finite, 3 = essential */
    std::vector<std::pair<double, double>> A, B;
    for (int64_t i = 0; i < na; ++i)
      if ((group == 3) == bool(a[i].essential) && (group == 3 || a[i].dim == group))
        A.push_back({a[i].birth, a[i].death});
    for (int64_t i = 0; i < nb; ++i)
      if ((group == 3) == bool(b[i].essential) && (group == 3 || b[i].dim == group))
        B.push_back({b[i].birth, b[i].death});
    worst = std::max(worst, bottleneck_group(A, B));
  }
  *out = worst;
  return 0;
}

int tso_simplify(const float* f, const int64_t dims[3], const tso_signal* sig,
                 const tso_options* opt, float* g_out, tso_report* rep, double* trace,
                 int64_t trace_cap) {
  const auto t0 = std::chrono::steady_clock::now();
  Grid g(dims);
  if (!g.valid || !f || !sig || !opt || !g_out || !rep) return -1;
  if (sig->mode == 1 && sig->n_signal > 0 && !sig->signal) return -1;
  if (!all_finite(f, g.n)) return -2;
  std::memset(rep, 0, sizeof(*rep));

  double fmin = f[0], fmax = f[0];
  for (int64_t i = 0; i < g.n; ++i) {
    fmin = std::min(fmin, double(f[i]));
    fmax = std::max(fmax, double(f[i]));
  }
  const double range = fmax - fmin;
  const double tol = double(opt->cancel_tol_rel) * range;

  std::vector<float> x(f, f + g.n);
  Persistence Pers;
  persistence(g, x.data(), &Pers);
  std::vector<Point> P = points_of(Pers.diagram);
  Solver S(g);
  std::vector<int> phi;
  S.build_targets(P, Pers.diagram, sig, range, &phi);
  const double L0 = S.loss(P, phi);
  double L = L0;
  if (trace && trace_cap > 0) trace[0] = L0;

  auto done = [&](double Lc) {
    if (opt->stop_mode == 1) return Lc <= double(opt->loss_ratio_s) * L0;
    return S.max_diag_pers(P, phi) < tol;
  };
  int j = 0;
  int64_t n_still = int64_t(P.size()), n_reduced = 0;
  bool cancelled = opt->stop_mode == 0 && done(L);
  while (!cancelled && j < opt->j_max) {
    ++j;
    S.step(&x, P, phi, opt->alpha_b, opt->alpha_d);
    persistence(g, x.data(), &Pers);
    std::vector<Point> Pn = points_of(Pers.diagram);
    std::vector<int> phin;
    S.assign(Pn, P, phi, &phin, &n_still, &n_reduced);
    P.swap(Pn);
    phi.swap(phin);
    L = S.loss(P, phi);
    if (trace && j < trace_cap) trace[j] = L;
    cancelled = done(L);
  }

  std::copy(x.begin(), x.end(), g_out);
  rep->iterations = j;
  rep->cancelled = cancelled ? 1 : 0;
  rep->loss0 = L0;
  rep->loss = L;
  rep->energy = L + S.unmatched_target_cost(phi);
  double linf = 0, l2 = 0;
  for (int64_t i = 0; i < g.n; ++i) {
    const double d = double(x[i]) - double(f[i]);
    linf = std::max(linf, std::fabs(d));
    l2 += d * d;
  }
  rep->linf = linf;
  rep->l2 = std::sqrt(l2);
  rep->max_nonsignal_pers = S.max_diag_pers(P, phi);
  double disp = 0;
  for (size_t i = 0; i < P.size(); ++i)
    if (phi[i] >= 0)
      disp = std::max(disp, std::sqrt(pair_cost(P[i].b, P[i].d, S.T[phi[i]].b, S.T[phi[i]].d)));
  rep->max_signal_disp = disp;
  rep->range = range;
  for (const Point& p : P)
    if (!p.essential) rep->n_pairs[p.dim]++;
  rep->n_still = n_still;
  rep->n_reduced = n_reduced;
  rep->n_targets = int64_t(S.T.size());
  rep->total_s =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return cancelled ? 0 : 1;
}

}  /* extern "C" */
