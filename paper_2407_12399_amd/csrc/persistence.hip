// persistence.hip -- the persistence map on gfx950 (Sec. 2.2 and 4.2).
//
//   K1/K2  vertex order: monotone 32-bit keys of (value), stable LSD radix
//          sort of (key, id) pairs, rank scatter.
//   K3     lower-star discrete gradient: one lane per vertex.  The cells of
//          the lower star are generated directly in lexicographic order
//          (grouped by their highest other vertex), so that both priority
//          queues of the lower-star algorithm become 128-bit masks over
//          sorted slots and "pop min" is a find-first-set.  Per vertex the
//          lane writes a 16-byte pairing code, its descending neighbour and
//          its critical cells with their lexicographic keys.
//   K4     critical cells: block-aggregated compaction inside K3, then a
//          radix sort per dimension by key.
//   K5     min-saddle pairs: critical edges join the minima their descending
//          paths reach; union-find over minima processed in rounds where
//          every component hooks to its lowest outgoing edge and the edges
//          that are the lowest outgoing edge of both their components merge
//          (those merges are exactly the next Kruskal steps, so the elder
//          rule applies to them as in the sequential sweep).
//   K6     saddle-max pairs: the same on the dual graph (tetrahedra and the
//          outside of the box) in decreasing order.
//   K7     saddle-saddle pairs: Morse boundaries of the remaining critical
//          triangles by mod-2 expansion along gradient paths, then a
//          parallel Z2 reduction (every column whose pivot is not its own
//          adds the column of the lowest owner of that pivot, in rounds).
//   K8     diagram: v_birth != v_death filter, diagram-order sort.
#include <mutex>
#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "persistence.h"

namespace ts {
namespace {

// ======================================================================
// Star tables of a vertex in the Freudenthal triangulation
// ======================================================================

struct StarTables {
  int8_t nb[14][3];          // neighbour offsets: k<7: +corner(k+1), k>=7: -corner(k-6)
  uint16_t tri_nbm[36];      // the two neighbours of star triangle t (14-bit mask)
  uint8_t tri_nb[36][2];
  uint16_t tet_nbm[24];      // the three neighbours of star tet q
  uint8_t tet_nb[24][3];
  uint64_t tet_trim[24];     // its three facets through the centre (36-bit mask)
  uint8_t tri_tet[36][2];    // the two star tets containing t
  uint64_t edge_trim[14];    // star triangles containing neighbour k
  uint32_t tri_tetm[36];     // star tets containing t (24-bit mask)
  uint8_t pair_tri[14][14];  // star triangle on neighbours (a,b), 255 if none
  int8_t tri_anc[36][3];     // anchor (lowest vertex) offset of the canonical cell
  uint8_t tri_type[36];
  int8_t tet_anc[24][3];
  uint8_t tet_type[24];
  uint8_t tri_local[12][3];  // canonical triangle type, chain position -> star index
  uint8_t tet_local[6][4];   // canonical tet type, chain position -> star index
  uint8_t tri_chain[12][3];  // corner masks of the canonical chains
  uint16_t negx, posx, negy, posy, negz, posz;  // neighbours leaving the box side
  int8_t nb_diff[14][14];    // star index of offset nb[b] - nb[a], -1 if not a neighbour
  // expansion step of the Morse boundary: edge (centre, k) paired with its
  // j-th star triangle (centre, k, k2): bit 31 valid, bits 0..3 k2, 4..7
  // nb_diff[k][k2], 8..11 nb_diff[k2][k]
  uint32_t edge_step[14][6];
};

__constant__ StarTables c_st;

// Canonical Kuhn chains (corner masks, bit0 = x, bit1 = y, bit2 = z).
const int kTriChains[12][3] = {{0, 1, 3}, {0, 2, 3}, {0, 1, 5}, {0, 4, 5},
                               {0, 2, 6}, {0, 4, 6}, {0, 1, 7}, {0, 2, 7},
                               {0, 3, 7}, {0, 4, 7}, {0, 5, 7}, {0, 6, 7}};
const int kTetChains[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7},
                              {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};

struct V3 {
  int x, y, z;
};
V3 corner3(int m) { return {m & 1, (m >> 1) & 1, (m >> 2) & 1}; }

int nb_of_offset(V3 d) {
  const bool pos = d.x >= 0 && d.y >= 0 && d.z >= 0;
  const bool neg = d.x <= 0 && d.y <= 0 && d.z <= 0;
  if (pos) {
    const int m = d.x | (d.y << 1) | (d.z << 2);
    return m == 0 ? -1 : m - 1;
  }
  if (neg) {
    const int m = (-d.x) | ((-d.y) << 1) | ((-d.z) << 2);
    return 7 + m - 1;
  }
  return -1;
}

// If the offsets (relative to the centre, which is included as (0,0,0)) form
// a Kuhn simplex, returns its anchor offset, canonical type and the corner
// masks of the points relative to the anchor.
bool kuhn_cell(const std::vector<V3>& pts, V3* anc, int* type) {
  V3 a = pts[0];
  for (const V3& p : pts) {
    a.x = std::min(a.x, p.x);
    a.y = std::min(a.y, p.y);
    a.z = std::min(a.z, p.z);
  }
  std::vector<int> masks;
  for (const V3& p : pts) {
    const int dx = p.x - a.x, dy = p.y - a.y, dz = p.z - a.z;
    if (dx > 1 || dy > 1 || dz > 1) return false;
    masks.push_back(dx | (dy << 1) | (dz << 2));
  }
  std::sort(masks.begin(), masks.end(),
            [](int u, int v) { return __builtin_popcount(u) < __builtin_popcount(v); });
  if (masks[0] != 0) return false;
  for (size_t i = 1; i < masks.size(); ++i)
    if ((masks[i - 1] & masks[i]) != masks[i - 1] || masks[i - 1] == masks[i]) return false;
  *anc = a;
  const int dim = int(pts.size()) - 1;
  if (dim == 2) {
    for (int t = 0; t < 12; ++t)
      if (kTriChains[t][1] == masks[1] && kTriChains[t][2] == masks[2]) {
        *type = t;
        return true;
      }
    return false;
  }
  for (int t = 0; t < 6; ++t)
    if (kTetChains[t][1] == masks[1] && kTetChains[t][2] == masks[2] && masks[3] == 7) {
      *type = t;
      return true;
    }
  return false;
}

StarTables build_tables() {
  StarTables T;
  std::memset(&T, 0, sizeof(T));
  std::memset(T.pair_tri, 255, sizeof(T.pair_tri));
  std::memset(T.tri_tet, 255, sizeof(T.tri_tet));
  V3 nb[14];
  for (int k = 0; k < 14; ++k) {
    V3 c = corner3(k % 7 + 1);
    if (k >= 7) c = {-c.x, -c.y, -c.z};
    nb[k] = c;
    T.nb[k][0] = int8_t(c.x);
    T.nb[k][1] = int8_t(c.y);
    T.nb[k][2] = int8_t(c.z);
    if (c.x < 0) T.negx |= 1u << k;
    if (c.x > 0) T.posx |= 1u << k;
    if (c.y < 0) T.negy |= 1u << k;
    if (c.y > 0) T.posy |= 1u << k;
    if (c.z < 0) T.negz |= 1u << k;
    if (c.z > 0) T.posz |= 1u << k;
  }
  for (int a = 0; a < 14; ++a)
    for (int b = 0; b < 14; ++b) {
      const V3 d = {nb[b].x - nb[a].x, nb[b].y - nb[a].y, nb[b].z - nb[a].z};
      T.nb_diff[a][b] = -1;
      for (int k = 0; k < 14; ++k)
        if (nb[k].x == d.x && nb[k].y == d.y && nb[k].z == d.z) T.nb_diff[a][b] = int8_t(k);
    }
  int nt = 0;
  for (int a = 0; a < 14; ++a)
    for (int b = a + 1; b < 14; ++b) {
      V3 anc;
      int type;
      if (!kuhn_cell({{0, 0, 0}, nb[a], nb[b]}, &anc, &type)) continue;
      if (nt >= 36) throw Error(TS_ERR_INTERNAL, "star tables: too many triangles");
      T.tri_nb[nt][0] = uint8_t(a);
      T.tri_nb[nt][1] = uint8_t(b);
      T.tri_nbm[nt] = uint16_t((1u << a) | (1u << b));
      T.pair_tri[a][b] = T.pair_tri[b][a] = uint8_t(nt);
      T.tri_anc[nt][0] = int8_t(anc.x);
      T.tri_anc[nt][1] = int8_t(anc.y);
      T.tri_anc[nt][2] = int8_t(anc.z);
      T.tri_type[nt] = uint8_t(type);
      T.edge_trim[a] |= 1ull << nt;
      T.edge_trim[b] |= 1ull << nt;
      ++nt;
    }
  int nq = 0;
  for (int a = 0; a < 14; ++a)
    for (int b = a + 1; b < 14; ++b)
      for (int c = b + 1; c < 14; ++c) {
        V3 anc;
        int type;
        if (!kuhn_cell({{0, 0, 0}, nb[a], nb[b], nb[c]}, &anc, &type)) continue;
        if (nq >= 24) throw Error(TS_ERR_INTERNAL, "star tables: too many tets");
        T.tet_nb[nq][0] = uint8_t(a);
        T.tet_nb[nq][1] = uint8_t(b);
        T.tet_nb[nq][2] = uint8_t(c);
        T.tet_nbm[nq] = uint16_t((1u << a) | (1u << b) | (1u << c));
        T.tet_anc[nq][0] = int8_t(anc.x);
        T.tet_anc[nq][1] = int8_t(anc.y);
        T.tet_anc[nq][2] = int8_t(anc.z);
        T.tet_type[nq] = uint8_t(type);
        const int tris[3] = {T.pair_tri[a][b], T.pair_tri[a][c], T.pair_tri[b][c]};
        for (int i = 0; i < 3; ++i) {
          const int t = tris[i];
          if (t == 255) throw Error(TS_ERR_INTERNAL, "star tables: tet facet missing");
          T.tet_trim[nq] |= 1ull << t;
          T.tri_tetm[t] |= 1u << nq;
          if (T.tri_tet[t][0] == 255) T.tri_tet[t][0] = uint8_t(nq);
          else T.tri_tet[t][1] = uint8_t(nq);
        }
        ++nq;
      }
  if (nt != 36 || nq != 24) throw Error(TS_ERR_INTERNAL, "star tables: wrong star size");
  for (int t = 0; t < 36; ++t)
    if (T.tri_tet[t][1] == 255) throw Error(TS_ERR_INTERNAL, "star tables: open triangle");
  for (int k = 0; k < 14; ++k)  // edge codes 0..5 name one of at most 6 triangles
    if (__builtin_popcountll(T.edge_trim[k]) > 6)
      throw Error(TS_ERR_INTERNAL, "star tables: edge of degree > 6");
  for (int k = 0; k < 14; ++k) {
    uint64_t m = T.edge_trim[k];
    for (int j = 0; j < 6; ++j) {
      T.edge_step[k][j] = 0;
      if (m == 0) continue;
      const int t = __builtin_ctzll(m);
      m &= m - 1;
      const int k2 = __builtin_ctz(uint32_t(T.tri_nbm[t]) & ~(1u << k));
      if (T.nb_diff[k][k2] < 0 || T.nb_diff[k2][k] < 0)
        throw Error(TS_ERR_INTERNAL, "star tables: triangle edge is not a neighbour offset");
      T.edge_step[k][j] = (1u << 31) | uint32_t(k2) | (uint32_t(T.nb_diff[k][k2]) << 4) |
                          (uint32_t(T.nb_diff[k2][k]) << 8);
    }
  }
  // canonical cell -> star index at each of its vertices
  for (int type = 0; type < 12; ++type) {
    for (int k = 0; k < 3; ++k) T.tri_chain[type][k] = uint8_t(kTriChains[type][k]);
    for (int p = 0; p < 3; ++p) {
      const V3 c = corner3(kTriChains[type][p]);
      int ks[2], m = 0;
      for (int q = 0; q < 3; ++q)
        if (q != p) {
          const V3 o = corner3(kTriChains[type][q]);
          ks[m++] = nb_of_offset({o.x - c.x, o.y - c.y, o.z - c.z});
        }
      const int t = T.pair_tri[ks[0]][ks[1]];
      if (t == 255) throw Error(TS_ERR_INTERNAL, "star tables: triangle inverse");
      T.tri_local[type][p] = uint8_t(t);
    }
  }
  for (int type = 0; type < 6; ++type)
    for (int p = 0; p < 4; ++p) {
      const V3 c = corner3(kTetChains[type][p]);
      uint32_t m = 0;
      for (int q = 0; q < 4; ++q)
        if (q != p) {
          const V3 o = corner3(kTetChains[type][q]);
          m |= 1u << nb_of_offset({o.x - c.x, o.y - c.y, o.z - c.z});
        }
      int found = -1;
      for (int l = 0; l < 24; ++l)
        if (T.tet_nbm[l] == m) found = l;
      if (found < 0) throw Error(TS_ERR_INTERNAL, "star tables: tet inverse");
      T.tet_local[type][p] = uint8_t(found);
    }
  return T;
}

void upload_tables(int device) {
  static bool done[64] = {false};
  if (device >= 0 && device < 64 && done[device]) return;
  static const StarTables T = build_tables();
  TS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_st), &T, sizeof(T)));
  if (device >= 0 && device < 64) done[device] = true;
}

// ======================================================================
// Device helpers
// ======================================================================

struct NbOff {
  int o[14];
};

NbOff make_offsets(const Grid& g) {
  NbOff r;
  for (int k = 0; k < 14; ++k) {
    V3 c = corner3(k % 7 + 1);
    if (k >= 7) c = {-c.x, -c.y, -c.z};
    r.o[k] = c.x + g.Lx * (c.y + g.Ly * c.z);
  }
  return r;
}

__device__ __forceinline__ void coords(const Grid& g, int v, int* x, int* y, int* z) {
  const int t = v / g.Lx;
  *x = v - t * g.Lx;
  *y = t % g.Ly;
  *z = t / g.Ly;
}

__device__ __forceinline__ uint32_t valid_nbs(const Grid& g, int x, int y, int z) {
  uint32_t m = 0x3FFFu;
  if (x == 0) m &= ~uint32_t(c_st.negx);
  if (x == g.Lx - 1) m &= ~uint32_t(c_st.posx);
  if (y == 0) m &= ~uint32_t(c_st.negy);
  if (y == g.Ly - 1) m &= ~uint32_t(c_st.posy);
  if (z == 0) m &= ~uint32_t(c_st.negz);
  if (z == g.Lz - 1) m &= ~uint32_t(c_st.posz);
  return m;
}

__device__ __forceinline__ int lin(const Grid& g, int dx, int dy, int dz) {
  return dx + g.Lx * (dy + g.Ly * dz);
}

// ---- field geometry ----
// Kernels that walk the grid see it through a geometry provider: site(v)
// gives the grid of the field holding vertex v (local coordinates, validity of
// the 14 neighbours, linear steps, neighbour offsets).  Vertex and cell ids
// stay global, so arrays are indexed as for one grid.
//   GeoOne:   one field; grid and offsets are kernel arguments.
//   GeoBatch: fields stored one after another, field f at [base, base + n);
//             a page map gives the field of each 2^kPageBits-vertex page's
//             first vertex, and a short forward scan finds v's field.
constexpr int kPageBits = 10;

struct FieldDesc {
  int base;  // first vertex of the field in the batch
  int Lx, Ly, Lz;
  int o[14];  // neighbour offsets
};

struct SiteOne {
  const Grid& g;
  const NbOff& off;
  __device__ __forceinline__ void xyz(int v, int* x, int* y, int* z) const { coords(g, v, x, y, z); }
  __device__ __forceinline__ uint32_t valid_at(int x, int y, int z) const {
    return valid_nbs(g, x, y, z);
  }
  __device__ __forceinline__ int step(int dx, int dy, int dz) const { return lin(g, dx, dy, dz); }
  __device__ __forceinline__ int nb(int k) const { return off.o[k]; }
};

struct SiteBatch {
  Grid g;  // the field's grid (n unused)
  int base;
  const int* o;
  __device__ __forceinline__ void xyz(int v, int* x, int* y, int* z) const {
    coords(g, v - base, x, y, z);
  }
  __device__ __forceinline__ uint32_t valid_at(int x, int y, int z) const {
    return valid_nbs(g, x, y, z);
  }
  __device__ __forceinline__ int step(int dx, int dy, int dz) const { return lin(g, dx, dy, dz); }
  __device__ __forceinline__ int nb(int k) const { return o[k]; }
};

struct GeoOne {
  Grid g;
  NbOff off;
  __device__ __forceinline__ int total() const { return g.n; }
  __device__ __forceinline__ SiteOne site(int) const { return SiteOne{g, off}; }
};

struct GeoBatch {
  const FieldDesc* fd;
  const int32_t* page;
  int nf;
  int n;  // vertices of the whole batch
  __device__ __forceinline__ int total() const { return n; }
  __device__ __forceinline__ int field(int v) const {
    int f = page[v >> kPageBits];
    while (f + 1 < nf && v >= fd[f + 1].base) ++f;
    return f;
  }
  __device__ __forceinline__ SiteBatch site(int v) const {
    const FieldDesc* F = fd + field(v);
    SiteBatch s;
    s.g.Lx = F->Lx;
    s.g.Ly = F->Ly;
    s.g.Lz = F->Lz;
    s.g.n = F->Lx * F->Ly * F->Lz;
    s.base = F->base;
    s.o = F->o;
    return s;
  }
};

__device__ __forceinline__ uint32_t nib(uint64_t packed, int i) {
  return uint32_t(packed >> (4 * i)) & 15u;
}

// code layout: w0,w1[0:10) = 14 edge codes of 3 bits; w1[10:18) = triangle
// codes 32..35; w1[18:32) = lower-neighbour mask (bit k: neighbour k is in
// the grid and precedes the vertex in the order); w2,w3 = triangle codes
// 0..31 (2 bits each).
//   edge code: 0..5 paired with the j-th star triangle containing the edge,
//              6 critical, 7 paired with the centre vertex
//   triangle code: 0 paired with a facet (or not in the lower star),
//              1 critical, 2/3 paired with tri_tet[t][0/1]
__device__ __forceinline__ uint32_t edge_code(const uint4& c, int k) {
  const uint64_t e = uint64_t(c.x) | (uint64_t(c.y & 0x3FFu) << 32);
  return uint32_t(e >> (3 * k)) & 7u;
}
__device__ __forceinline__ uint32_t lower_mask(const uint4& c) { return c.y >> 18; }
__device__ __forceinline__ uint32_t tri_code(const uint4& c, int t) {
  if (t < 32) {
    const uint64_t e = uint64_t(c.z) | (uint64_t(c.w) << 32);
    return uint32_t(e >> (2 * t)) & 3u;
  }
  return (c.y >> (10 + 2 * (t - 32))) & 3u;
}

__device__ __forceinline__ int ffs64(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int ffs32(uint32_t m) { return __ffs(m) - 1; }

// ======================================================================
// K1 / K2: vertex order
// ======================================================================

__global__ void k_order_keys(const float* __restrict__ f, int n, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ vals, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t b = __float_as_uint(f[i]);
  if ((b & 0x7F800000u) == 0x7F800000u) atomicOr(bad, 1);  // NaN or Inf
  if ((b & 0x7FFFFFFFu) == 0u) b = 0u;                     // -0 -> +0
  keys[i] = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  vals[i] = uint32_t(i);
}

__global__ void k_rank_scatter(const uint32_t* __restrict__ order, int n, int32_t* __restrict__ rank,
                               int32_t* __restrict__ order_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = order[i];
  rank[v] = i;
  if (order_out) order_out[i] = int32_t(v);
}

// ======================================================================
// K3: lower-star gradient
// ======================================================================

struct CritOut {
  uint64_t* key[4];
  int32_t* id[4];
  unsigned long long* count;  // [4]
  int64_t cap[4];
};

constexpr int kGradThreads = 256;
constexpr int kSlotBytes = 74;  // >= 74 lower-star cells (excluding the centre)
constexpr int kCellBytes = 74;  // 14 edges, 36 triangles, 24 tets

// The star tables that the lower-star loop indexes per lane, staged in LDS
// (lane-dependent indices into constant memory become vector-memory loads).
struct HotTables {
  uint64_t tet_trim[24];
  uint64_t edge_trim[14];
  uint32_t tri_tetm[36];
  uint16_t tri_nbm[36];
  uint16_t tet_nbm[24];
  uint8_t tri_tet[36][2];
  uint8_t pair_tri[14][14];
  // the two star tets on triangle t and the neighbour each adds to it:
  // bytes (tet 0, its third neighbour, tet 1, its third neighbour)
  uint32_t tri_info[36];
  // neighbours b with a star triangle on (k, b) (14-bit mask)
  uint16_t edge_adj[14];
};

// LDS of the lower-star kernel: per-lane slot tables and the block's
// emission counters.
struct K3Shared {
  __align__(16) uint8_t slot_cell[kSlotBytes * kGradThreads];
  __align__(16) uint8_t cell_slot[kCellBytes * kGradThreads];
  unsigned int cnt[4];
  unsigned long long base[4];
};

__device__ __forceinline__ void load_hot_tables(HotTables& T) {
  const int tid = threadIdx.x;
  if (tid < 24) T.tet_trim[tid] = c_st.tet_trim[tid];
  if (tid < 14) T.edge_trim[tid] = c_st.edge_trim[tid];
  if (tid < 36) {
    T.tri_tetm[tid] = c_st.tri_tetm[tid];
    T.tri_nbm[tid] = c_st.tri_nbm[tid];
    T.tri_tet[tid][0] = c_st.tri_tet[tid][0];
    T.tri_tet[tid][1] = c_st.tri_tet[tid][1];
    uint32_t info = 0;
    for (int i = 0; i < 2; ++i) {
      const uint32_t q = c_st.tri_tet[tid][i];
      const uint32_t c = uint32_t(ffs32(uint32_t(c_st.tet_nbm[q]) & ~uint32_t(c_st.tri_nbm[tid])));
      info |= (q | (c << 8)) << (16 * i);
    }
    T.tri_info[tid] = info;
  }
  if (tid < 24) T.tet_nbm[tid] = c_st.tet_nbm[tid];
  if (tid < 14) {
    uint32_t adj = 0;
    for (int b = 0; b < 14; ++b)
      if (c_st.pair_tri[tid][b] != 255) adj |= 1u << b;
    T.edge_adj[tid] = uint16_t(adj);
  }
  if (tid < 196) T.pair_tri[tid / 14][tid % 14] = c_st.pair_tri[tid / 14][tid % 14];
}

// One block's worth of lower stars: lane tid brings vertex v0 (act0: a vertex
// to process).  kWaveMode false: called by every thread of the block (it holds
// barriers: the block's vertices are sorted by work first, and the critical
// cells are emitted with one atomic per block).  kWaveMode true: the lane's
// vertex is processed as given and the cells are emitted with one atomic per
// wave, with no barrier, so that the waves of a block run independently.
template <bool kWaveMode = false, class Geo>
__device__ __forceinline__ void k3_block(const int32_t* __restrict__ rank, const Geo& G,
                                         uint4* __restrict__ code_out,
                                         int32_t* __restrict__ down_out, const CritOut& co,
                                         const HotTables& T, K3Shared& sh, bool act0, int v0) {
  const int tid = threadIdx.x;
  uint8_t* s_slot_cell = sh.slot_cell;
  uint8_t* s_cell_slot = sh.cell_slot;
  unsigned int* s_cnt = sh.cnt;
  unsigned long long* s_base = sh.base;
  if (!kWaveMode && tid < 4) s_cnt[tid] = 0;
  uint8_t* slot_cell = s_slot_cell + tid;  // element i at [i * kGradThreads]
  uint8_t* cell_slot = s_cell_slot + tid;
#define SLOT_CELL(i) slot_cell[(i) * kGradThreads]
#define CELL_SLOT(i) cell_slot[(i) * kGradThreads]

  // The lower-star loops run as often as the slowest lane of a wave needs, and
  // their trip counts grow with the number of lower neighbours.  The block's
  // vertices are therefore first sorted by that number (a counting sort in
  // LDS, in the space the slot tables use later), so that each wave holds
  // vertices of similar work.  Every output is indexed by vertex, so the
  // processing order does not change any result.
  int v = v0;
  bool active = act0;
  if constexpr (!kWaveMode) {
    int key = 15;  // inactive lanes last
    if (act0) {
      const auto S0 = G.site(v0);
      int x, y, z;
      S0.xyz(v0, &x, &y, &z);
      const uint32_t valid = S0.valid_at(x, y, z);
      const int r0 = rank[v0];
      int c = 0;
#pragma unroll
      for (int k = 0; k < 14; ++k)
        if ((valid >> k) & 1u) c += rank[v0 + S0.nb(k)] < r0 ? 1 : 0;
      key = c;
    }
    unsigned int* s_hist = reinterpret_cast<unsigned int*>(s_cell_slot);  // 16 counters
    int* s_sorted = reinterpret_cast<int*>(s_slot_cell);                 // kGradThreads vertices
    if (tid < 16) s_hist[tid] = 0;
    __syncthreads();
    const unsigned int within = atomicAdd(&s_hist[key], 1u);
    __syncthreads();
    if (tid == 0) {
      unsigned int acc = 0;
      for (int b = 0; b < 16; ++b) {
        const unsigned int t = s_hist[b];
        s_hist[b] = acc;
        acc += t;
      }
    }
    __syncthreads();
    s_sorted[s_hist[key] + within] = act0 ? v0 : -1;
    __syncthreads();
    const int mine = s_sorted[tid];
    __syncthreads();  // the slot tables reuse this space below
    active = mine >= 0;
    v = active ? mine : 0;
  }
  const auto S = G.site(active ? v : 0);
  int rx = 0;
  uint32_t low = 0;
  // nibble k: position of neighbour k among the lower neighbours, 15 for a
  // neighbour that is not lower
  uint64_t pos = 0;
  uint32_t critE = 0, critQ = 0;
  uint64_t critT = 0;
  uint64_t ecode = 0;          // 3 bits per neighbour
  uint64_t tcode0 = 0;         // 2 bits per triangle 0..31
  uint32_t tcode1 = 0;         // triangles 32..35
  if (active) {
    int x, y, z;
    S.xyz(v, &x, &y, &z);
    const uint32_t valid = S.valid_at(x, y, z);
    rx = rank[v];
    int r[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      r[k] = INT_MAX;
      if ((valid >> k) & 1u) {
        r[k] = rank[v + S.nb(k)];
        if (r[k] < rx) low |= 1u << k;
      }
    }
    // position of lower neighbour k = the number of neighbours of lower rank
    // (the others, and missing ones at INT_MAX, rank above it), counted once
    // per pair: p[j] starts at the 13 - j pairs (j, k > j) and loses those
    // where r[j] is the larger; ranks are distinct, so this is exact wherever
    // r[j] ties with no other rank, that is for every lower neighbour
    uint32_t pk[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) pk[k] = uint32_t(13 - k);
#pragma unroll
    for (int k = 1; k < 14; ++k)
#pragma unroll
      for (int j = 0; j < k; ++j) {
        const uint32_t c = r[j] < r[k] ? 1u : 0u;
        pk[k] += c;
        pk[j] -= c;
      }
    uint64_t bypos = 0;  // nibble p: neighbour at position p
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      const bool lk = (low >> k) & 1u;
      pos |= uint64_t(lk ? pk[k] : 15u) << (4 * k);
      if (lk) bypos |= uint64_t(k) << (4 * pk[k]);
    }
    if (low == 0) {
      down_out[v] = v;
    } else {
      const int k0 = int(nib(bypos, 0));
      down_out[v] = v + S.nb(k0);
      uint32_t Lq = 0;  // lower tets
#pragma unroll
      for (int q = 0; q < 24; ++q)
        if ((uint32_t(T.tet_nbm[q]) & low) == uint32_t(T.tet_nbm[q])) Lq |= 1u << q;

      // lower-star cells in lexicographic order: by highest other vertex P,
      // then the triangle (P,Q) for increasing Q followed by its tets (P,Q,R)
      // for increasing R
      const int cnt = __popc(low);
      int s = 0;
      uint64_t eslot0 = 0, eslot1 = 0;
      for (int P = 0; P < cnt; ++P) {
        const int a = int(nib(bypos, P));
        SLOT_CELL(s) = uint8_t((1u << 6) | a);
        CELL_SLOT(a) = uint8_t(s);
        if (s < 64) eslot0 |= 1ull << s;
        else eslot1 |= 1ull << (s - 64);
        ++s;
        for (int Q = 0; Q < P; ++Q) {
          const int b = int(nib(bypos, Q));
          const int t = T.pair_tri[a][b];
          if (t == 255) continue;
          SLOT_CELL(s) = uint8_t((2u << 6) | t);
          CELL_SLOT(14 + t) = uint8_t(s);
          ++s;
          // tets on triangle t whose third neighbour is lower than b (a
          // neighbour that is not lower has position 15 > Q), by increasing
          // position of that neighbour
          const uint32_t ti = T.tri_info[t];
          const uint32_t q0 = ti & 255u, q1 = (ti >> 16) & 255u;
          const uint32_t r0 = nib(pos, int((ti >> 8) & 255u)), r1 = nib(pos, int(ti >> 24));
          const bool in0 = r0 < uint32_t(Q), in1 = r1 < uint32_t(Q);
          int qa = -1, qb = -1;
          if (in0 && in1) {
            qa = int(r0 < r1 ? q0 : q1);
            qb = int(r0 < r1 ? q1 : q0);
          } else if (in0) {
            qa = int(q0);
          } else if (in1) {
            qa = int(q1);
          }
          if (qa >= 0) {
            SLOT_CELL(s) = uint8_t((3u << 6) | qa);
            CELL_SLOT(50 + qa) = uint8_t(s);
            ++s;
          }
          if (qb >= 0) {
            SLOT_CELL(s) = uint8_t((3u << 6) | qb);
            CELL_SLOT(50 + qb) = uint8_t(s);
            ++s;
          }
        }
      }

      uint32_t Ec = 1u << k0, Qc = 0;
      uint64_t Tc = 0;
      uint64_t O0 = 0, O1 = 0, Z0 = eslot0 & ~1ull, Z1 = eslot1;
      ecode |= 7ull << (3 * k0);

      auto set_slot = [&](uint64_t& m0, uint64_t& m1, int sl) {
        if (sl < 64) m0 |= 1ull << sl;
        else m1 |= 1ull << (sl - 64);
      };
      // edge k was just paired (k is in Ec): a lower triangle (k, b) now has
      // one unpaired face exactly when edge b is unpaired
      auto push_edge_cof = [&](int k) {
        uint32_t m = uint32_t(T.edge_adj[k]) & low & ~Ec;
        while (m) {
          const int b = ffs32(m);
          m &= m - 1;
          set_slot(O0, O1, CELL_SLOT(14 + T.pair_tri[k][b]));
        }
      };
      // triangle t was just paired: of its two star tets, the lower ones left
      // with one unpaired face
      auto push_tri_cof = [&](int t) {
        const uint32_t ti = T.tri_info[t];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int q = int((ti >> (16 * i)) & 255u);
          if (((Lq >> q) & 1u) && __popcll(T.tet_trim[q] & ~Tc) == 1)
            set_slot(O0, O1, CELL_SLOT(50 + q));
        }
      };
      auto set_tcode = [&](int t, uint32_t c) {
        if (t < 32) tcode0 |= uint64_t(c) << (2 * t);
        else tcode1 |= c << (2 * (t - 32));
      };

      push_edge_cof(k0);
      for (;;) {
        while (O0 | O1) {
          int sl;
          if (O0) {
            sl = ffs64(O0);
            O0 &= O0 - 1;
          } else {
            sl = 64 + ffs64(O1);
            O1 &= O1 - 1;
          }
          const uint32_t cc = SLOT_CELL(sl);
          const int dim = int(cc >> 6), idx = int(cc & 63u);
          // a triangle pairs with its unpaired edge, a tet with its unpaired
          // triangle; then the paired triangle's tets (and the paired edge's
          // triangles) are pushed, once for both kinds
          int tri = -1, edge = -1;
          if (dim == 2) {
            if ((Tc >> idx) & 1ull) continue;
            const uint32_t u = uint32_t(T.tri_nbm[idx]) & ~Ec;
            if (u == 0) {
              set_slot(Z0, Z1, sl);
              continue;
            }
            const int k = ffs32(u);
            Ec |= 1u << k;
            Tc |= 1ull << idx;
            const uint32_t j = __popcll(T.edge_trim[k] & ((1ull << idx) - 1ull));
            ecode |= uint64_t(j) << (3 * k);
            tri = idx;
            edge = k;
          } else {
            if ((Qc >> idx) & 1u) continue;
            const uint64_t u = T.tet_trim[idx] & ~Tc;
            if (u == 0) {
              set_slot(Z0, Z1, sl);
              continue;
            }
            const int t = ffs64(u);
            Tc |= 1ull << t;
            Qc |= 1u << idx;
            set_tcode(t, T.tri_tet[t][0] == idx ? 2u : 3u);
            tri = t;
          }
          push_tri_cof(tri);
          if (edge >= 0) push_edge_cof(edge);
        }
        if (!(Z0 | Z1)) break;
        int sl;
        if (Z0) {
          sl = ffs64(Z0);
          Z0 &= Z0 - 1;
        } else {
          sl = 64 + ffs64(Z1);
          Z1 &= Z1 - 1;
        }
        const uint32_t cc = SLOT_CELL(sl);
        const int dim = int(cc >> 6), idx = int(cc & 63u);
        if (dim == 1) {
          if ((Ec >> idx) & 1u) continue;
          Ec |= 1u << idx;
          critE |= 1u << idx;
          ecode |= 6ull << (3 * idx);
          push_edge_cof(idx);
        } else if (dim == 2) {
          if ((Tc >> idx) & 1ull) continue;
          Tc |= 1ull << idx;
          critT |= 1ull << idx;
          set_tcode(idx, 1u);
          push_tri_cof(idx);
        } else {
          if ((Qc >> idx) & 1u) continue;
          Qc |= 1u << idx;
          critQ |= 1u << idx;
        }
      }
    }
    uint4 c;
    c.x = uint32_t(ecode);
    c.y = uint32_t(ecode >> 32) | (tcode1 << 10) | (low << 18);
    c.z = uint32_t(tcode0);
    c.w = uint32_t(tcode0 >> 32);
    code_out[v] = c;
  }
#undef SLOT_CELL
#undef CELL_SLOT

  // ---- emit critical cells (block-aggregated) ----
  const unsigned int nv = (active && low == 0) ? 1u : 0u;
  const unsigned int ne = __popc(critE), nt = __popcll(critT), nq = __popc(critQ);
  unsigned long long p0, p1, p2, p3;  // first output slot of each kind
  if constexpr (kWaveMode) {
    // exclusive prefix of each kind's count over the wave, one atomic a kind
    const unsigned lane = threadIdx.x & 63u;
    auto reserve = [&](unsigned int c, unsigned long long* counter) {
      unsigned int incl = c;
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned int y = unsigned(__shfl_up(int(incl), d, 64));
        if (int(lane) >= d) incl += y;
      }
      const unsigned int tot = unsigned(__shfl(int(incl), 63, 64));
      unsigned long long b = 0;
      if (lane == 63 && tot) b = atomicAdd(counter, (unsigned long long)tot);
      b = __shfl(b, 63, 64);
      return b + (incl - c);
    };
    p0 = reserve(nv, &co.count[0]);
    p1 = reserve(ne, &co.count[1]);
    p2 = reserve(nt, &co.count[2]);
    p3 = reserve(nq, &co.count[3]);
  } else {
    __syncthreads();
    unsigned int o0 = 0, o1 = 0, o2 = 0, o3 = 0;
    if (nv) o0 = atomicAdd(&s_cnt[0], nv);
    if (ne) o1 = atomicAdd(&s_cnt[1], ne);
    if (nt) o2 = atomicAdd(&s_cnt[2], nt);
    if (nq) o3 = atomicAdd(&s_cnt[3], nq);
    __syncthreads();
    if (tid < 4) s_base[tid] = s_cnt[tid] ? atomicAdd(&co.count[tid], (unsigned long long)s_cnt[tid]) : 0ull;
    __syncthreads();
    p0 = s_base[0] + o0;
    p1 = s_base[1] + o1;
    p2 = s_base[2] + o2;
    p3 = s_base[3] + o3;
  }
  if (!active) return;
  const uint64_t rk = uint64_t(rx) << 12;
  if (nv) {
    const unsigned long long p = p0;
    if ((int64_t)p < co.cap[0]) {
      co.key[0][p] = rk;
      co.id[0][p] = v;
    }
  }
  if (ne) {
    unsigned long long p = p1;
    uint32_t m = critE;
    while (m) {
      const int k = ffs32(m);
      m &= m - 1;
      if ((int64_t)p < co.cap[1]) {
        const int anchor = k < 7 ? v : v + S.nb(k);
        co.key[1][p] = rk | (uint64_t(nib(pos, k) + 1) << 8);
        co.id[1][p] = 7 * anchor + (k % 7);
      }
      ++p;
    }
  }
  if (nt) {
    unsigned long long p = p2;
    uint64_t m = critT;
    while (m) {
      const int t = ffs64(m);
      m &= m - 1;
      if ((int64_t)p < co.cap[2]) {
        const uint32_t pa = nib(pos, c_st.tri_nb[t][0]), pb = nib(pos, c_st.tri_nb[t][1]);
        const uint32_t hi = max(pa, pb), lo = min(pa, pb);
        const int anchor = v + S.step(c_st.tri_anc[t][0], c_st.tri_anc[t][1], c_st.tri_anc[t][2]);
        co.key[2][p] = rk | (uint64_t(hi + 1) << 8) | (uint64_t(lo + 1) << 4);
        co.id[2][p] = 12 * anchor + c_st.tri_type[t];
      }
      ++p;
    }
  }
  if (nq) {
    unsigned long long p = p3;
    uint32_t m = critQ;
    while (m) {
      const int q = ffs32(m);
      m &= m - 1;
      if ((int64_t)p < co.cap[3]) {
        uint32_t a = nib(pos, c_st.tet_nb[q][0]), b = nib(pos, c_st.tet_nb[q][1]),
                 c = nib(pos, c_st.tet_nb[q][2]);
        // sort descending
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        if (b < c) { const uint32_t t = b; b = c; c = t; }
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const int anchor = v + S.step(c_st.tet_anc[q][0], c_st.tet_anc[q][1], c_st.tet_anc[q][2]);
        co.key[3][p] = rk | (uint64_t(a + 1) << 8) | (uint64_t(b + 1) << 4) | uint64_t(c + 1);
        co.id[3][p] = 6 * anchor + c_st.tet_type[q];
      }
      ++p;
    }
  }
}

// kList: lane i processes vertex vlist[i] (i < nlist) instead of vertex i.
template <bool kList, class Geo>
__global__ void __launch_bounds__(kGradThreads)
k_gradient(const int32_t* __restrict__ rank, Geo G, uint4* __restrict__ code_out,
           int32_t* __restrict__ down_out, CritOut co, const uint32_t* __restrict__ vlist,
           int64_t nlist) {
  __shared__ K3Shared sh;
  __shared__ HotTables T;
  load_hot_tables(T);
  __syncthreads();
  const int64_t lane = int64_t(blockIdx.x) * kGradThreads + threadIdx.x;
  const bool act0 = kList ? lane < nlist : lane < G.total();
  const int v0 = kList ? (act0 ? int(vlist[lane]) : 0) : int(lane);
  k3_block(rank, G, code_out, down_out, co, T, sh, act0, v0);
}

// Work queue of 3D tiles for the persistent form of the lower-star kernel: the
// tiles of field f are items tile_base[f] .. tile_base[f + 1] - 1, numbered x
// fastest within the field; a tile holds tx * ty * tz = kGradThreads vertices,
// with tx and ty powers of two.
// tx == 0 instead makes item i the run of vertex ids i * kGradThreads ..
// (i + 1) * kGradThreads - 1 over all fields (no idle lanes at field edges).
// The items are split into kTileQueues contiguous ranges, one queue each;
// workgroup b starts on queue b % kTileQueues, which keeps it on one XCD's
// slab of the grid (workgroups are dealt to the 8 XCDs in turn), so that
// neighbouring tiles share that XCD's L2 for their halos and partly written
// lines; a workgroup whose queue is empty moves on to the next ones.
constexpr int kTileQueues = 8;
struct TileQueue {
  const int4* field;          // per field: (base vertex, Lx, Ly, Lz)
  const int64_t* tile_base;   // nf + 1 prefix counts of tiles
  int nf;
  int tx, ty, tz;
  unsigned int* head;         // kTileQueues counters (cleared before the launch)
  int64_t nitems;
  __device__ int64_t begin(int qi) const { return nitems * qi / kTileQueues; }
};

// The lower-star kernel as persistent workgroups that take tiles from a
// queue until it is empty: the hot tables are staged once per workgroup, and a
// tile keeps the 14-neighbour stencil of its vertices within a small box.
// A workgroup takes two tiles at a time (512 vertices), sorts them by their
// number of lower neighbours (the lower-star loops run as often as a wave's
// slowest lane needs, and their trip counts grow with that number), and its
// waves then take the eight groups of 64 sorted vertices from a shared
// counter, the heaviest first, each emitting its own critical cells: a wave
// that drew light groups takes more of them instead of waiting at a barrier
// for the wave with the heaviest one.
constexpr int kK3Batch = 2;  // tiles per workgroup round
template <class Geo>
__global__ void __launch_bounds__(kGradThreads)
k_gradient_tiles(const int32_t* __restrict__ rank, Geo G, uint4* __restrict__ code_out,
                 int32_t* __restrict__ down_out, CritOut co, TileQueue q) {
  __shared__ K3Shared sh;
  __shared__ HotTables T;
  __shared__ int64_t s_item[kK3Batch];
  // per item of the round: (first vertex, vertices of the field left from
  // the tile's corner along x, y and z) and the field's y and z strides
  __shared__ int4 s_tile[kK3Batch];
  __shared__ int2 s_stride[kK3Batch];
  __shared__ uint16_t s_order[kK3Batch * kGradThreads];  // batch slots sorted by work
  __shared__ unsigned int s_hist[16];
  __shared__ int s_next;
  load_hot_tables(T);
  const int tid = threadIdx.x;
  const unsigned lane = threadIdx.x & 63u;
  const bool runs = q.tx == 0;
  // lane position -> tile coordinates (tile sides are powers of two; a run is
  // one row of kGradThreads)
  const int sx = ffs32(uint32_t(runs ? kGradThreads : q.tx)), sy = runs ? 0 : ffs32(uint32_t(q.ty));
  const int mx = (1 << sx) - 1, my = (1 << sy) - 1;
  // the corner and extent of item `item` (once per item, on one lane)
  auto place = [&](int b, int64_t item) {
    int4 t = make_int4(0, 0, 0, 0);  // no item: no lane is inside
    int2 st = make_int2(0, 0);
    if (item >= 0 && runs) {
      const int64_t v0 = item * kGradThreads;
      t = make_int4(int(v0), int(min<int64_t>(G.total() - v0, kGradThreads)), 1, 1);
    } else if (item >= 0) {
      int f = 0;
      while (f + 1 < q.nf && item >= q.tile_base[f + 1]) ++f;
      const int4 fd = q.field[f];
      const int nbx = (fd.y + q.tx - 1) / q.tx, nby = (fd.z + q.ty - 1) / q.ty;
      const int64_t i = item - q.tile_base[f];
      const int bx = int(i % nbx), by = int((i / nbx) % nby), bz = int(i / (int64_t(nbx) * nby));
      const int x = bx * q.tx, y = by * q.ty, z = bz * q.tz;
      t = make_int4(fd.x + x + fd.y * (y + fd.z * z), fd.y - x, fd.z - y, fd.w - z);
      st = make_int2(fd.y, fd.y * fd.z);
    }
    s_tile[b] = t;
    s_stride[b] = st;
  };
  // vertex of lane position `pos` of the round's item b (act: inside its field)
  auto vertex = [&](int b, int pos, bool* act) -> int {
    const int4 t = s_tile[b];
    const int2 st = s_stride[b];
    const int lx = pos & mx, ly = (pos >> sx) & my, lz = pos >> (sx + sy);
    *act = lx < t.y && ly < t.z && lz < t.w;
    return *act ? t.x + lx + st.x * ly + st.y * lz : 0;
  };
  int probe = 0;  // queues tried so far (uniform over the workgroup)
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      for (int b = 0; b < kK3Batch; ++b) {
        s_item[b] = -1;
        for (; probe < kTileQueues; ++probe) {
          const int qi = int((blockIdx.x + probe) % kTileQueues);
          const int64_t i = q.begin(qi) + int64_t(atomicAdd(q.head + qi, 1u));
          if (i < q.begin(qi + 1)) {
            s_item[b] = i;
            break;
          }
        }
        place(b, s_item[b]);
      }
      s_next = 0;
    }
    if (tid < 16) s_hist[tid] = 0;
    __syncthreads();
    if (s_item[0] < 0) break;  // the whole workgroup leaves together
    // sort the batch's vertices by their number of lower neighbours (vertices
    // outside the grid count as 0, with the cheapest)
    int key[kK3Batch];
    unsigned int within[kK3Batch];
#pragma unroll
    for (int b = 0; b < kK3Batch; ++b) {
      bool act;
      const int v = vertex(b, tid, &act);
      int c = 0;
      if (act) {
        const auto S0 = G.site(v);
        int x, y, z;
        S0.xyz(v, &x, &y, &z);
        const uint32_t valid = S0.valid_at(x, y, z);
        const int r0 = rank[v];
#pragma unroll
        for (int k = 0; k < 14; ++k)
          if ((valid >> k) & 1u) c += rank[v + S0.nb(k)] < r0 ? 1 : 0;
      }
      key[b] = c;
      within[b] = atomicAdd(&s_hist[c], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      unsigned int acc = 0;
      for (int b = 0; b < 16; ++b) {
        const unsigned int t = s_hist[b];
        s_hist[b] = acc;
        acc += t;
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kK3Batch; ++b)
      s_order[s_hist[key[b]] + within[b]] = uint16_t(b * kGradThreads + tid);
    __syncthreads();
    constexpr int kGroups = kK3Batch * kGradThreads / 64;
    for (;;) {
      // keep the LDS table reads inside the loop (hoisted, they would hold
      // a hundred registers and cost a wave per SIMD)
      asm volatile("" ::: "memory");
      int g = 0;
      if (lane == 0) g = atomicAdd(&s_next, 1);
      g = __shfl(g, 0, 64);
      if (g >= kGroups) break;
      const int slot = s_order[(kGroups - 1 - g) * 64 + int(lane)];  // heaviest first
      bool act;
      const int v = vertex(slot / kGradThreads, slot % kGradThreads, &act);
      k3_block<true>(rank, G, code_out, down_out, co, T, sh, act, v);
    }
  }
}

// ---- fast update of the gradient between solver iterations (Sec. 4.2) ----
// The lower star of v, hence its gradient code, its descent step and its
// critical cells (up to the rank prefix of their keys), depends only on the
// relative order of v and its 14 neighbours.  Unchanged values keep their
// relative order, so only vertices with a changed value in their closed star
// (dirty vertices) need the lower-star loop again.

// Stream compaction in a 256-lane block: each lane handles kAppendPer items
// (round j covers items base + j * 256 + lane).  Lanes record per round their
// wave's count in s_cnt[j * 4 + wave]; block_reserve turns the counts into
// offsets and reserves the block's range with one atomic, so items land in
// (round, wave, lane) order and the counter sees one atomic per block.
constexpr int kAppendPer = 16;

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ void block_reserve(unsigned int* s_cnt, unsigned long long* counter,
                              unsigned long long* s_base) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const unsigned int c = s_cnt[lane];
    unsigned int x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned int y = unsigned(__shfl_up(int(x), d, 64));
      if (lane >= d) x += y;
    }
    s_cnt[lane] = x - c;
    if (lane == 63) *s_base = x ? atomicAdd(counter, (unsigned long long)x) : 0ull;
  }
  __syncthreads();
}

// dirty[v] = v or a neighbour changed value; dirty vertices are appended to
// list and counted in *count.
template <class Geo>
__global__ void __launch_bounds__(256)
k_dirty(const uint8_t* __restrict__ changed, Geo G, uint8_t* __restrict__ dirty,
        uint32_t* __restrict__ list, unsigned long long* __restrict__ count) {
  __shared__ unsigned int s_cnt[4 * kAppendPer];
  __shared__ unsigned long long s_base;
  const int wave = threadIdx.x >> 6;
  const int64_t base = int64_t(blockIdx.x) * 256 * kAppendPer + threadIdx.x;
  uint32_t bits = 0;
#pragma unroll 1
  for (int j = 0; j < kAppendPer; ++j) {
    const int64_t i = base + j * 256;
    bool d = false;
    if (i < G.total()) {
      const int v = int(i);
      const auto S = G.site(v);
      int x, y, z;
      S.xyz(v, &x, &y, &z);
      const uint32_t valid = S.valid_at(x, y, z);
      uint32_t c = changed[v];
#pragma unroll
      for (int k = 0; k < 14; ++k)
        if ((valid >> k) & 1u) c |= changed[v + S.nb(k)];
      d = c != 0;
      dirty[v] = d ? 1 : 0;
    }
    bits |= uint32_t(d) << j;
    const uint64_t m = __ballot(d);
    if (__lane_id() == 0) s_cnt[j * 4 + wave] = unsigned(__popcll(m));
  }
  block_reserve(s_cnt, count, &s_base);
#pragma unroll 1
  for (int j = 0; j < kAppendPer; ++j) {
    const bool d = (bits >> j) & 1u;
    const uint64_t m = __ballot(d);
    if (d) list[s_base + s_cnt[j * 4 + wave] + __popcll(m & lanes_below())] = uint32_t(base + j * 256);
  }
}

// Critical cells of the previous map whose highest vertex is clean, with the
// key prefix replaced by that vertex's new rank.  prev_order maps the old
// rank prefix back to the vertex.  Appends at count (bounded by cap).
__global__ void __launch_bounds__(256)
k_keep_crit(const uint64_t* __restrict__ pkey, const int32_t* __restrict__ pid, int64_t np,
            const int32_t* __restrict__ prev_order, const int32_t* __restrict__ rank,
            const uint8_t* __restrict__ dirty, uint64_t* __restrict__ key,
            int32_t* __restrict__ id, int64_t cap, unsigned long long* __restrict__ count) {
  __shared__ unsigned int s_cnt[4 * kAppendPer];
  __shared__ unsigned long long s_base;
  const int wave = threadIdx.x >> 6;
  const int64_t base = int64_t(blockIdx.x) * 256 * kAppendPer + threadIdx.x;
  uint32_t bits = 0;
#pragma unroll 1
  for (int j = 0; j < kAppendPer; ++j) {
    const int64_t i = base + j * 256;
    bool keep = false;
    if (i < np) keep = dirty[prev_order[pkey[i] >> 12]] == 0;
    bits |= uint32_t(keep) << j;
    const uint64_t m = __ballot(keep);
    if (__lane_id() == 0) s_cnt[j * 4 + wave] = unsigned(__popcll(m));
  }
  block_reserve(s_cnt, count, &s_base);
#pragma unroll 1
  for (int j = 0; j < kAppendPer; ++j) {
    const bool keep = (bits >> j) & 1u;
    const uint64_t m = __ballot(keep);
    if (!keep) continue;
    const int64_t i = base + j * 256;
    const uint64_t pk = pkey[i];
    const int v = prev_order[pk >> 12];
    const unsigned long long p = s_base + s_cnt[j * 4 + wave] + __popcll(m & lanes_below());
    if ((int64_t)p < cap) {
      key[p] = (uint64_t(uint32_t(rank[v])) << 12) | (pk & 0xFFFull);
      id[p] = pid[i];
    }
  }
}

// ======================================================================
// Lookup helpers
// ======================================================================

__global__ void k_set_marks(unsigned int* __restrict__ mark, int64_t n,
                            const unsigned int* __restrict__ round_ptr) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) mark[i] = *round_ptr;
}

__global__ void k_iota_from(uint32_t* a, int64_t n, uint32_t base) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = base + uint32_t(i);
}

// sort keys that order a list of columns by decreasing index
__global__ void k_desc_keys(const uint32_t* __restrict__ list, int64_t n, uint32_t top,
                            uint32_t* __restrict__ keys) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = top - list[i];
}

__global__ void k_iota(uint32_t* a, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = uint32_t(i);
}

__global__ void k_gather_ids(const int32_t* __restrict__ ids, const uint32_t* __restrict__ perm,
                             int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = uint32_t(ids[perm[i]]);
}

// index of `id` in the id-sorted array, -1 if absent
// pos_of[id] = position of the critical cell with canonical id `id` in its
// key-sorted list (entries of non-critical ids are never read)
__global__ void k_pos_map(const int32_t* __restrict__ ids, int64_t m, int32_t* __restrict__ pos_of) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) pos_of[ids[i]] = int32_t(i);
}

// After the D0 pairing: the position of a critical edge that dies in
// dimension 0 (state != 1) becomes -1 - position, so that the saddle-saddle
// boundary drops such an edge after one load.
__global__ void k_pos_drop(const int32_t* __restrict__ ids, const uint8_t* __restrict__ state,
                           int64_t m, int32_t* __restrict__ pos_of) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m && state[i] != 1) pos_of[ids[i]] = int32_t(-1 - i);
}

// position of critical cell `id` (checked against the list), -1 if not critical
__device__ __forceinline__ int64_t crit_pos(const int32_t* __restrict__ pos_of,
                                            const int32_t* __restrict__ ids, int64_t m, int id) {
  const int32_t p = pos_of[id];
  return (p >= 0 && p < m && ids[p] == id) ? p : -1;
}


// ======================================================================
// K5: min-saddle pairs
// ======================================================================

__global__ void k_min_index(const int32_t* __restrict__ min_ids, int64_t nmin,
                            int32_t* __restrict__ min_idx) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nmin) min_idx[min_ids[i]] = int32_t(i);
}

// endpoints of critical edge i -> components (indices of the minima reached)
template <class Geo>
__global__ void k_d0_init(const int32_t* __restrict__ edge_ids, int64_t ne, Geo G,
                          const int32_t* __restrict__ down, const int32_t* __restrict__ min_idx,
                          int32_t* __restrict__ ca, int32_t* __restrict__ cb,
                          uint32_t* __restrict__ list, int* __restrict__ err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  const int id = edge_ids[i];
  const int u = id / 7, t = id - 7 * (id / 7);
  const int m = t + 1;
  const int w = u + G.site(u).step(m & 1, (m >> 1) & 1, (m >> 2) & 1);
  int ends[2] = {u, w};
  int comp[2];
  for (int e = 0; e < 2; ++e) {
    int a = ends[e];
    int steps = 0;
    while (true) {
      const int d = down[a];
      if (d == a) break;
      a = d;
      if (++steps > G.total()) {
        atomicOr(err, 1);
        break;
      }
    }
    comp[e] = min_idx[a];
  }
  ca[i] = comp[0];
  cb[i] = comp[1];
  list[i] = uint32_t(i);
}

// Slot of this thread's item in a list appended to by whole blocks: one
// atomic per block on the list counter (per-wave atomics on one counter
// serialise tens of thousands of operations when millions of items are
// appended).  Every thread of the block calls it, once per kernel; blocks of
// at most 1024 threads.  The order of the list is unspecified.
template <class C>
__device__ __forceinline__ C block_append(bool take, C* counter) {
  __shared__ unsigned int s_wcnt[16];
  __shared__ C s_base;
  const uint64_t m = __ballot(take);
  const int lane = __lane_id();
  const int wave = int(threadIdx.x >> 6);
  if (lane == 0) s_wcnt[wave] = unsigned(__popcll(m));
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int tot = 0;
    for (int w = 0; w < int((blockDim.x + 63) >> 6); ++w) tot += s_wcnt[w];
    s_base = tot ? atomicAdd(counter, C(tot)) : C(0);
  }
  __syncthreads();
  C b = s_base;
  for (int w = 0; w < wave; ++w) b += s_wcnt[w];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  return b + C(__popcll(m & lt));
}

// Union-find with the elder rule, in rounds.  Every component finds its
// lowest outgoing edge (hook); then every component whose lowest outgoing
// edge leads to a component with an older representative joins it, and its
// representative dies at that edge (link).  That is the sequential sweep's
// decision: any path from the representative to an older node leaves its
// component through an edge no lower than the lowest outgoing one, and the
// other side reaches its older representative through edges no higher than
// it.  prio(i) = i (increasing order) or nedges-1-i (decreasing order).
__device__ __forceinline__ int uf_find(int32_t* parent, int x) {
  while (true) {
    const int p = parent[x];
    if (p == x) return x;
    const int gp = parent[p];
    if (gp != p) parent[x] = gp;  // path halving (any ancestor is a valid parent)
    x = gp;
  }
}

__global__ void k_uf_hook(const uint32_t* __restrict__ list, const unsigned int* __restrict__ nlist,
                          int32_t* __restrict__ ca, int32_t* __restrict__ cb,
                          int32_t* __restrict__ parent, unsigned int* __restrict__ best,
                          uint8_t* __restrict__ state, int descending, int64_t nedges) {
  const unsigned int j = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned int n = *nlist;
  if (j >= n) return;
  // the list holds edges in about increasing index order; visit them in about
  // increasing priority (reversed for the descending order), so that a
  // component's lowest edge tends to come first and the plain read below
  // filters out the later ones (the result does not depend on the order)
  const uint32_t i = list[descending ? n - 1 - j : j];
  const int a = uf_find(parent, ca[i]), b = uf_find(parent, cb[i]);
  ca[i] = a;
  cb[i] = b;
  if (a == b) {
    state[i] = 1;  // closes a cycle: no merge
    return;
  }
  const unsigned int pr = descending ? unsigned(nedges - 1 - i) : i;
  // best[] of a large component is hit by many edges: a plain read filters
  // out most of the atomics (best only decreases within a round)
  if (pr < best[a]) atomicMin(&best[a], pr);
  if (pr < best[b]) atomicMin(&best[b], pr);
}

struct PairOut {
  int32_t* dim;
  int32_t* birth;
  int32_t* death;
  uint64_t* bkey;
  uint64_t* dkey;
  unsigned long long* count;
  int64_t cap;
};

//   dual == 0: nodes are minima by increasing key (smaller index = older);
//              pair (min, edge)
//   dual == 1: nodes are maxima by increasing key and the outside (index
//              nnodes-1); larger index = older; pair (triangle, max tet)
__global__ void k_uf_link(const uint32_t* __restrict__ list, const unsigned int* __restrict__ nlist,
                          const int32_t* __restrict__ ca, const int32_t* __restrict__ cb,
                          int32_t* __restrict__ parent, const unsigned int* __restrict__ best,
                          uint8_t* __restrict__ state, uint32_t* __restrict__ next,
                          unsigned int* __restrict__ nnext, int dual, int64_t nedges,
                          const int32_t* __restrict__ cell_id, const uint64_t* __restrict__ cell_key,
                          const int32_t* __restrict__ node_id, const uint64_t* __restrict__ node_key,
                          PairOut po) {
  const unsigned int j = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t i = 0;
  int younger = 0, elder = 0;
  bool link = false, keep = false;
  if (j < *nlist) {
    i = list[j];
    if (state[i] == 0) {
      const int a = ca[i], b = cb[i];
      const unsigned int pr = dual ? unsigned(nedges - 1 - i) : i;
      // the younger endpoint component may join the older one along its lowest edge
      const bool a_older = dual ? (a > b) : (a < b);
      younger = a_older ? b : a;
      elder = a_older ? a : b;
      link = best[younger] == pr;
      keep = !link;
    }
  }
  // the kept edges (millions in the first rounds) are appended per block, the
  // pairs (fewer) per wave
  const unsigned int q = block_append(keep, nnext);
  const uint64_t ml = __ballot(link);
  const int lane = __lane_id();
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long pb = 0;
  if (lane == 0 && ml) pb = atomicAdd(po.count, (unsigned long long)__popcll(ml));
  pb = (unsigned long long)__shfl((long long)pb, 0, 64);
  if (keep) next[q] = i;
  if (link) {
    parent[younger] = elder;
    state[i] = 2;
    const unsigned long long p = pb + __popcll(ml & lt);
    if ((int64_t)p < po.cap) {
      if (!dual) {
        po.dim[p] = 0;
        po.birth[p] = node_id[younger];
        po.death[p] = cell_id[i];
        po.bkey[p] = node_key[younger];
        po.dkey[p] = cell_key[i];
      } else {
        po.dim[p] = 2;
        po.birth[p] = cell_id[i];
        po.death[p] = node_id[younger];
        po.bkey[p] = cell_key[i];
        po.dkey[p] = node_key[younger];
      }
    }
  }
}

__global__ void k_uf_reset(int32_t* __restrict__ parent, unsigned int* __restrict__ best,
                           int64_t nnodes) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nnodes) return;
  best[c] = 0xFFFFFFFFu;
  uf_find(parent, int(c));
}

__global__ void k_uf_init(int32_t* __restrict__ parent, unsigned int* __restrict__ best,
                          int64_t nnodes) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nnodes) return;
  best[c] = 0xFFFFFFFFu;
  parent[c] = int32_t(c);
}

// ======================================================================
// K6: saddle-max pairs (ascending gradient paths)
// ======================================================================

// Follows the ascending gradient path from star tet l of vertex y to a
// maximum; returns the canonical id of the maximum, or -1 for the outside.
template <class Site>
__device__ int ascend(const Site& S, int total, const uint4* __restrict__ code, int y, int l,
                      int* err) {
  int steps = 0;
  while (true) {
    if (++steps > 6 * total) {
      atomicOr(err, 2);
      return -1;
    }
    const uint4 c = code[y];
    int paired_t = -1, side = 0;
    uint64_t fm = c_st.tet_trim[l];
    while (fm) {
      const int t = ffs64(fm);
      fm &= fm - 1;
      const uint32_t tc = tri_code(c, t);
      if (tc >= 2 && c_st.tri_tet[t][tc - 2] == l) {
        paired_t = t;
        side = int(tc - 2);
      }
    }
    if (paired_t < 0) {
      const int anchor = y + S.step(c_st.tet_anc[l][0], c_st.tet_anc[l][1], c_st.tet_anc[l][2]);
      return 6 * anchor + c_st.tet_type[l];
    }
    const int other = c_st.tri_tet[paired_t][1 - side];
    const uint32_t third = uint32_t(c_st.tet_nbm[other]) & ~uint32_t(c_st.tri_nbm[paired_t]);
    const int k = ffs32(third);
    int x, yy, z;
    S.xyz(y, &x, &yy, &z);
    const uint32_t valid = S.valid_at(x, yy, z);
    if (!((valid >> k) & 1u)) return -1;  // the facet lies on the box boundary
    const int cv = y + S.nb(k);
    if ((lower_mask(c) >> k) & 1u) {  // cv precedes y: the tet stays in y's lower star
      l = other;
    } else {
      // the next tet belongs to the lower star of its new apex cv
      const int anchor =
          y + S.step(c_st.tet_anc[other][0], c_st.tet_anc[other][1], c_st.tet_anc[other][2]);
      const int type = c_st.tet_type[other];
      int ax, ay, az, cx, cy, cz;
      S.xyz(anchor, &ax, &ay, &az);
      S.xyz(cv, &cx, &cy, &cz);
      const int mask = (cx - ax) | ((cy - ay) << 1) | ((cz - az) << 2);
      l = c_st.tet_local[type][__popc(mask)];
      y = cv;
    }
  }
}

template <class Geo>
__global__ void k_d2_init(const int32_t* __restrict__ tri_ids, const uint64_t* __restrict__ tri_keys,
                          int64_t nt, Geo G, const int32_t* __restrict__ order,
                          const uint4* __restrict__ code,
                          const int32_t* __restrict__ max_pos_of,
                          const int32_t* __restrict__ max_ids, int64_t nmax,
                          int32_t* __restrict__ ca, int32_t* __restrict__ cb,
                          uint32_t* __restrict__ list, int* __restrict__ err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const int id = tri_ids[i];
  const int y = order[tri_keys[i] >> 12];  // highest vertex of the triangle
  const auto S = G.site(y);
  const int anchor = id / 12, type = id - 12 * (id / 12);
  int ax, ay, az, cx, cy, cz;
  S.xyz(anchor, &ax, &ay, &az);
  S.xyz(y, &cx, &cy, &cz);
  const int mask = (cx - ax) | ((cy - ay) << 1) | ((cz - az) << 2);
  const int p = mask == 0 ? 0 : (mask == c_st.tri_chain[type][1] ? 1 : 2);
  const int lt = c_st.tri_local[type][p];
  int x, yy, z;
  S.xyz(y, &x, &yy, &z);
  const uint32_t valid = S.valid_at(x, yy, z);
  const uint32_t lowy = lower_mask(code[y]);
  int comp[2];
  for (int s = 0; s < 2; ++s) {
    const int q = c_st.tri_tet[lt][s];
    if ((uint32_t(c_st.tet_nbm[q]) & valid) != uint32_t(c_st.tet_nbm[q])) {
      comp[s] = int(nmax);  // outside of the box
      continue;
    }
    // the tet is in the lower star of y unless its third vertex is higher
    const uint32_t third = uint32_t(c_st.tet_nbm[q]) & ~uint32_t(c_st.tri_nbm[lt]);
    const int k = ffs32(third);
    const int cv = y + S.nb(k);
    int yv = y, l = q;
    if (!((lowy >> k) & 1u)) {  // cv follows y
      const int anc = y + S.step(c_st.tet_anc[q][0], c_st.tet_anc[q][1], c_st.tet_anc[q][2]);
      const int qt = c_st.tet_type[q];
      int bx, by, bz, vx, vy, vz;
      S.xyz(anc, &bx, &by, &bz);
      S.xyz(cv, &vx, &vy, &vz);
      const int m2 = (vx - bx) | ((vy - by) << 1) | ((vz - bz) << 2);
      l = c_st.tet_local[qt][__popc(m2)];
      yv = cv;
    }
    const int mid = ascend(S, G.total(), code, yv, l, err);
    if (mid < 0) {
      comp[s] = int(nmax);
    } else {
      const int64_t f = crit_pos(max_pos_of, max_ids, nmax, mid);
      if (f < 0) {
        atomicOr(err, 4);
        comp[s] = int(nmax);
      } else {
        comp[s] = int(f);
      }
    }
  }
  ca[i] = comp[0];
  cb[i] = comp[1];
  list[i] = uint32_t(i);
}

// ======================================================================
// K7: saddle-saddle pairs
// ======================================================================

// Per-lane scratch with an interleaved layout: element j of lane t lives at
// [j * stride + t], so that the lanes of a wave touching the same depth hit
// the same cache lines.
// Max-heap of edge keys (duplicates allowed), 4-ary: half the levels of a
// binary heap, and the four children of a node are loaded together, so a pop
// or push waits on about half as many dependent memory round trips.
struct LaneHeap {
  uint64_t* key;
  uint32_t* ref;
  int64_t stride;
  int len, cap;
  __device__ static bool leader() { return true; }
  __device__ void clear() { len = 0; }
  __device__ int size() const { return len; }
  __device__ uint64_t top_key() const { return key[0]; }
  __device__ uint32_t top_ref() const { return ref[0]; }
  __device__ uint64_t k(int j) const { return key[int64_t(j) * stride]; }
  __device__ bool push(uint64_t kk, uint32_t rr) {
    if (len >= cap) return false;
    int i = len++;
    while (i > 0) {
      const int p = (i - 1) >> 2;
      const uint64_t pk = k(p);
      if (pk >= kk) break;
      key[int64_t(i) * stride] = pk;
      ref[int64_t(i) * stride] = ref[int64_t(p) * stride];
      i = p;
    }
    key[int64_t(i) * stride] = kk;
    ref[int64_t(i) * stride] = rr;
    return true;
  }
  __device__ void pop(uint64_t* kk, uint32_t* rr) {
    *kk = key[0];
    *rr = ref[0];
    --len;
    if (len == 0) return;
    const uint64_t lk = k(len);
    const uint32_t lr = ref[int64_t(len) * stride];
    int i = 0;
    while (true) {
      const int c0 = 4 * i + 1;
      if (c0 >= len) break;
      uint64_t ck[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ck[j] = c0 + j < len ? k(c0 + j) : 0ull;
      int c = c0;
      uint64_t best = ck[0];
#pragma unroll
      for (int j = 1; j < 4; ++j)
        if (c0 + j < len && ck[j] > best) {
          best = ck[j];
          c = c0 + j;
        }
      if (best <= lk) break;
      key[int64_t(i) * stride] = best;
      ref[int64_t(i) * stride] = ref[int64_t(c) * stride];
      i = c;
    }
    key[int64_t(i) * stride] = lk;
    ref[int64_t(i) * stride] = lr;
  }
};

// toggle r in the ascending row list rows[0..*len) (interleaved); false on overflow
__device__ __forceinline__ bool toggle_row(uint32_t* rows, int64_t stride, int* len, int cap,
                                           uint32_t r, int* moved) {
  int lo = 0, hi = *len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rows[int64_t(mid) * stride] < r) lo = mid + 1;
    else hi = mid;
  }
  *moved += *len - lo;
  if (lo < *len && rows[int64_t(lo) * stride] == r) {
    for (int i = lo; i + 1 < *len; ++i) rows[int64_t(i) * stride] = rows[int64_t(i + 1) * stride];
    --*len;
    return true;
  }
  if (*len >= cap) return false;
  for (int i = *len; i > lo; --i) rows[int64_t(i) * stride] = rows[int64_t(i - 1) * stride];
  rows[int64_t(lo) * stride] = r;
  ++*len;
  return true;
}

struct ColPool {
  uint32_t* data;
  unsigned long long* top;
  int64_t cap;
};

struct BoundaryCommon {
  const uint32_t* cols;
  const int32_t* tri_ids;
  const uint64_t* tri_keys;
  const int32_t* rank;
  const int32_t* order;
  const uint4* code;
  const int32_t* edge_pos_of;  // canonical edge id -> position among critical edges
                               // (-1 - position for those that die in dimension 0)
  const int32_t* edge_ids;     // critical edge ids by position
  int64_t nedges;
  ColPool pool;
  uint64_t* col_desc;
  uint32_t* retry;
  unsigned int* nretry;
  int* pool_full;
  int* err;
  unsigned long long* stats;
  int max_steps;
  int wave_cap;   // queue capacity of the wave kernel's first pass (<= 256)
  int wave2_cap;  // and of its second pass (<= 1024)
};

template <class Geo>
struct BoundaryArgs : BoundaryCommon {
  Geo G;
};

// Morse boundary of critical triangle column c (mod 2, restricted to the
// critical edges that do not die in dimension 0), written descending: the
// expansion pops the highest edge of the multiset, cancels equal copies in
// pairs, and replaces an edge paired with a triangle by that triangle's two
// other edges.  An edge is (key = rank(h) << 32 | rank(o), ref = h << 4 | k)
// with h the higher vertex and k the star index of o.  A column whose heap or
// row list overflows, or that needs more than max_steps pops, is appended to
// the retry list and left unwritten.
// Cross-lane moves of the wave queue: DPP wave shifts (lane i takes lane
// i + 1, or i - 1) with the lane that has no source taking `in`, and reads of
// one lane's value.
__device__ __forceinline__ uint32_t wave_down(uint32_t v, uint32_t in) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(in), int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t wave_up(uint32_t v, uint32_t in) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(in), int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int lane) {
  return uint32_t(__builtin_amdgcn_readlane(int(v), lane));
}

// A max-priority queue of up to 64 R (key, ref) entries held by one wave in
// registers, as a sorted run in the physical slots i = 64 j + lane (R slots a
// lane): slots [0, off) are free, holding the all-ones key (above every edge
// key), slots [off, off + n) hold the entries sorted descending, and the
// slots after them key 0 (below every edge key).  Every lane makes every
// call, and the values returned are the same in all lanes.
//  - A pop reads slot off and frees it (off + 1); when the whole first
//    register is free, the registers move down by one.
//  - A push finds its place p with one ballot per register until the first
//    register that is not entirely above the new key.  If a free slot
//    precedes the run and p lies in the first register, the entries above
//    the new one move down by one slot (a single register, a few VALU
//    instructions): the common case of an expansion, whose first new edge
//    stays near the top.  Otherwise the entries after p move up by one,
//    register by register from the last occupied one down to p's, with the
//    carries across registers read from lane 63; registers entirely above p
//    are not touched.  When the slots run out while some are free, the run
//    is moved down to slot 0 first (cross-lane permutes).
template <int R>
struct WaveListR {
  static constexpr int kCap = 64 * R;
  uint32_t khi[R], klo[R], r[R];
  int n;    // entries
  int off;  // free slots before them (< 64)
  int lane;
  int cap = kCap;  // may be set lower (tests of the fallback)
  __device__ static bool leader() { return (threadIdx.x & 63) == 0; }
  __device__ static uint64_t join(uint32_t hi, uint32_t lo) { return (uint64_t(hi) << 32) | lo; }
  __device__ void clear() {
    lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < R; ++j) khi[j] = klo[j] = r[j] = 0;
    n = 0;
    off = 0;
  }
  __device__ int size() const { return n; }
  __device__ uint64_t top_key() const {
    return join(lane_value(khi[0], off), lane_value(klo[0], off));
  }
  __device__ uint32_t top_ref() const { return lane_value(r[0], off); }
  __device__ void pop(uint64_t* kk, uint32_t* rr) {
    *kk = top_key();
    *rr = top_ref();
    if (lane == off) khi[0] = klo[0] = ~0u;
    ++off;
    --n;
    if (n == 0) {  // empty: no free slots either (the later registers hold zeros)
      khi[0] = klo[0] = 0;
      off = 0;
    } else if (off == 64) {  // the first register is free: drop it
#pragma unroll
      for (int j = 0; j + 1 < R; ++j) {
        khi[j] = khi[j + 1];
        klo[j] = klo[j + 1];
        r[j] = r[j + 1];
      }
      khi[R - 1] = klo[R - 1] = r[R - 1] = 0;
      off = 0;
    }
  }
  // move the run down to slot 0 (slot i takes slot i + off)
  __device__ void compact() {
    const int src = lane + off, sl = src & 63;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t ah = __shfl(khi[j], sl), al = __shfl(klo[j], sl), ar = __shfl(r[j], sl);
      uint32_t bh = 0, bl = 0, br = 0;
      if (j + 1 < R) {
        bh = __shfl(khi[j + 1], sl);
        bl = __shfl(klo[j + 1], sl);
        br = __shfl(r[j + 1], sl);
      }
      khi[j] = src >= 64 ? bh : ah;
      klo[j] = src >= 64 ? bl : al;
      r[j] = src >= 64 ? br : ar;
    }
    off = 0;
  }
  __device__ bool push(uint64_t kk, uint32_t rr) {
    if (n >= cap) return false;
    int p = kCap;  // slots above the new entry (free slots count as above)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int c = __popcll(__ballot(join(khi[j], klo[j]) > kk));
      if (c < 64) {  // registers are sorted: the first one not entirely above
        p = 64 * j + c;
        break;
      }
    }
    if (off > 0 && p <= 64) {  // entries above move down into the free slot before them
      const uint32_t dh = wave_down(khi[0], 0u), dl = wave_down(klo[0], 0u),
                     dr = wave_down(r[0], 0u);
      if (lane >= off - 1 && lane < p - 1) {
        khi[0] = dh;
        klo[0] = dl;
        r[0] = dr;
      } else if (lane == p - 1) {
        khi[0] = uint32_t(kk >> 32);
        klo[0] = uint32_t(kk);
        r[0] = rr;
      }
      --off;
      ++n;
      return true;
    }
    if (off + n >= kCap) {  // no slot after the run: move it to slot 0 first
      p -= off;
      compact();
    }
    const int last = off + n;  // the slot of the last entry after the push
#pragma unroll
    for (int j = R - 1; j >= 0; --j) {  // slot i > p takes slot i - 1
      if (64 * j > last || 64 * j + 63 < p) continue;  // past the run, or entirely above p
      const uint32_t ch = j > 0 ? lane_value(khi[j - 1], 63) : 0u;
      const uint32_t cl = j > 0 ? lane_value(klo[j - 1], 63) : 0u;
      const uint32_t cr = j > 0 ? lane_value(r[j - 1], 63) : 0u;
      const uint32_t uh = wave_up(khi[j], ch), ul = wave_up(klo[j], cl), ur = wave_up(r[j], cr);
      const int i = 64 * j + lane;
      if (i > p) {
        khi[j] = uh;
        klo[j] = ul;
        r[j] = ur;
      } else if (i == p) {
        khi[j] = uint32_t(kk >> 32);
        klo[j] = uint32_t(kk);
        r[j] = rr;
      }
    }
    ++n;
    return true;
  }
};

// Neighbour ranks of a vertex group's higher vertex h, as the expansion of
// an edge (h, o) needs the rank of its third vertex, a lower neighbour of h.
// RanksDirect loads each when needed.  RanksWave loads the gradient code and
// the 14 neighbour ranks of a vertex in one round trip (lane j holds
// neighbour j; indices are clamped into the rank array and only the lower
// neighbours' ranks, which are in the grid, are used), and loads the next
// group's ahead (hint) while the current group is expanded.
template <class Site>
struct RanksDirect {
  const int32_t* rank;
  const uint4* code;
  Site S;
  int h = -1;
  __device__ RanksDirect(const int32_t* r, const uint4* c, const Site& s, int) : rank(r), code(c), S(s) {}
  __device__ uint4 start(int v) {
    h = v;
    return code[v];
  }
  __device__ uint32_t get(int k2) const { return uint32_t(rank[h + S.nb(k2)]); }
  __device__ void hint(int) {}
};

template <class Site>
struct RanksWave {
  const int32_t* rank;
  const uint4* code;
  Site S;
  int last;       // last index of the rank array
  uint32_t cur;   // this lane's neighbour rank of the current vertex
  int pf_v = -1;  // vertex loaded ahead
  uint4 pf_code;
  uint32_t pf_r;
  __device__ RanksWave(const int32_t* r, const uint4* c, const Site& s, int l)
      : rank(r), code(c), S(s), last(l) {}
  __device__ void load(int v) {
    const int lane = threadIdx.x & 63;
    int off = 0;
#pragma unroll
    for (int j = 0; j < 14; ++j)
      if (lane == j) off = S.nb(j);
    pf_v = v;
    pf_code = code[v];
    pf_r = uint32_t(rank[min(max(v + off, 0), last)]);
  }
  __device__ uint4 start(int v) {
    if (pf_v != v) load(v);
    cur = pf_r;
    pf_v = -1;
    return pf_code;
  }
  __device__ uint32_t get(int k2) const { return __shfl(cur, k2); }
  __device__ void hint(int v) {
    if (v != pf_v) load(v);
  }
};

template <bool kWave, class Q, class Geo, bool kLaneGroup = false>
__device__ __forceinline__ void boundary_column(const BoundaryArgs<Geo>& A, uint32_t c, Q& H,
                                                uint32_t* Rows, int64_t rstride, int rcap,
                                                uint32_t* Rk = nullptr) {
  const uint32_t ti = A.cols[c];
  const int id = A.tri_ids[ti];
  const int y = A.order[A.tri_keys[ti] >> 12];
  const auto S = A.G.site(y);  // the expansion stays in y's field
  const int anchor = id / 12, type = id - 12 * (id / 12);
  int ax, ay, az, cx, cy, cz;
  S.xyz(anchor, &ax, &ay, &az);
  S.xyz(y, &cx, &cy, &cz);
  const int mask = (cx - ax) | ((cy - ay) << 1) | ((cz - az) << 2);
  const int p = mask == 0 ? 0 : (mask == c_st.tri_chain[type][1] ? 1 : 2);
  const int lt = c_st.tri_local[type][p];
  const int ka = c_st.tri_nb[lt][0], kb = c_st.tri_nb[lt][1];
  H.clear();
  int rl = 0;
  // the three edges of the triangle (y is its highest vertex)
  const uint32_t ry = uint32_t(A.rank[y]);
  const uint32_t ra = uint32_t(A.rank[y + S.nb(ka)]), rb = uint32_t(A.rank[y + S.nb(kb)]);
  bool ok = H.push((uint64_t(ry) << 32) | ra, (uint32_t(y) << 4) | uint32_t(ka)) &&
            H.push((uint64_t(ry) << 32) | rb, (uint32_t(y) << 4) | uint32_t(kb));
  if (ok) {
    const bool a_hi = ra > rb;
    const int hv = y + S.nb(a_hi ? ka : kb);
    const int kk = c_st.nb_diff[a_hi ? ka : kb][a_hi ? kb : ka];
    ok = H.push((uint64_t(a_hi ? ra : rb) << 32) | (a_hi ? rb : ra), (uint32_t(hv) << 4) | uint32_t(kk));
  }
  int steps = 0, maxlen = H.size();
  int toggles = 0, moved = 0, groups = 0, expands = 0;  // diagnostics
  // edges leave the heap grouped by their higher vertex (it is the high part
  // of the key): the vertex's gradient code is loaded once per group
  int code_v = -1;
  uint4 code_h = make_uint4(0, 0, 0, 0);
  using Site = decltype(S);
  typename std::conditional<kWave, RanksWave<Site>, RanksDirect<Site>>::type N(
      A.rank, A.code, S, A.G.total() - 1);
  const bool lead = Q::leader();
  if constexpr (kWave) {
    // One vertex group at a time: the group's entries leave the queue
    // together, as a 14-bit set of star indices (mod 2: equal copies
    // cancel); the group is expanded inside that set, the highest-ranked
    // neighbour first (the order the queue would give them): an edge paired
    // with a star triangle (h, o, n2) flips n2 in the set and sends the edge
    // between o and n2, which belongs to a lower vertex, to the queue.
    const int ln = threadIdx.x & 63;
    while (ok && H.size() > 0) {
      maxlen = max(maxlen, H.size());
      const uint32_t rh = uint32_t(H.top_key() >> 32);
      const int h = int(H.top_ref() >> 4);
      uint32_t M = 0;
      while (H.size() > 0 && uint32_t(H.top_key() >> 32) == rh) {
        if (++steps > A.max_steps) {
          ok = false;
          break;
        }
        uint64_t kk;
        uint32_t rr;
        H.pop(&kk, &rr);
        M ^= 1u << (rr & 15u);
      }
      if (!ok) break;
      ++groups;
      code_h = N.start(h);
      if (H.size() > 0) N.hint(int(H.top_ref() >> 4));
      const uint32_t myrank = N.cur;  // lane j: rank of neighbour j
      while (M) {
        if (++steps > A.max_steps) {
          ok = false;
          break;
        }
        // the neighbour of highest rank in M (ranks are distinct)
        uint32_t v = (ln < 14 && ((M >> ln) & 1u)) ? myrank + 1u : 0u;
        v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xF, 0xF, false)));
        v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xF, 0xF, false)));
        v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xF, 0xF, false)));
        v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xF, 0xF, false)));
        const uint32_t top = lane_value(v, 15);
        const uint64_t at =
            __ballot(ln < 14 && ((M >> ln) & 1u) && myrank + 1u == top);
        if (at == 0) {  // cannot happen: M holds star indices below 14
          if (lead) atomicOr(A.err, 128);
          ok = false;
          break;
        }
        const int k = __ffsll((unsigned long long)at) - 1;
        M &= ~(1u << k);
        const uint32_t ec = edge_code(code_h, k);
        if (ec == 7u) continue;  // paired with its vertex: the path ends
        if (ec == 6u) {          // critical edge
          const int lo = h + S.nb(k);
          const int eid = k < 7 ? 7 * h + k : 7 * lo + (k - 7);
          const int32_t f = A.edge_pos_of[eid];
          if (f < 0 && int64_t(-1 - f) < A.nedges) continue;  // dies in dimension 0
          if (f < 0 || int64_t(f) >= A.nedges || A.edge_ids[f] != eid) {
            if (lead) atomicOr(A.err, 16);
            continue;
          }
          ++toggles;
          if (!toggle_row(Rows, rstride, &rl, rcap, uint32_t(f), &moved)) {
            ok = false;
            break;
          }
          continue;
        }
        const uint32_t stp = c_st.edge_step[k][ec];
        if (!(stp >> 31)) {
          if (lead) atomicOr(A.err, 128);
          ok = false;
          break;
        }
        const int k2 = int(stp & 15u);
        ++expands;
        M ^= 1u << k2;  // the edge (h, n2)
        const uint32_t ro = lane_value(myrank, k), rn = lane_value(myrank, k2);
        if (ro > rn) {
          ok = H.push((uint64_t(ro) << 32) | rn, (uint32_t(h + S.nb(k)) << 4) | ((stp >> 4) & 15u));
        } else {
          ok = H.push((uint64_t(rn) << 32) | ro, (uint32_t(h + S.nb(k2)) << 4) | ((stp >> 8) & 15u));
        }
      }
    }
  } else if constexpr (kLaneGroup) {
    // The same group expansion by one lane: the ranks of the set's members
    // (star index k -> rank) are kept in Rk[k * rstride] (LDS), and the
    // highest is found by a scan over the set, which holds a few members.
    while (ok && H.size() > 0) {
      maxlen = max(maxlen, H.size());
      const uint32_t rh = uint32_t(H.top_key() >> 32);
      const int h = int(H.top_ref() >> 4);
      uint32_t M = 0;
      while (H.size() > 0 && uint32_t(H.top_key() >> 32) == rh) {
        if (++steps > A.max_steps) {
          ok = false;
          break;
        }
        uint64_t kk;
        uint32_t rr;
        H.pop(&kk, &rr);
        const int kb = int(rr & 15u);
        M ^= 1u << kb;
        Rk[int64_t(kb) * rstride] = uint32_t(kk);
      }
      if (!ok) break;
      ++groups;
      code_h = N.start(h);
      while (M) {
        if (++steps > A.max_steps) {
          ok = false;
          break;
        }
        int k = -1;
        uint32_t ro = 0;
        for (uint32_t m = M; m; m &= m - 1) {
          const int b = __ffs(m) - 1;
          const uint32_t rb = Rk[int64_t(b) * rstride];
          if (k < 0 || rb > ro) {
            k = b;
            ro = rb;
          }
        }
        M &= ~(1u << k);
        const uint32_t ec = edge_code(code_h, k);
        if (ec == 7u) continue;  // paired with its vertex: the path ends
        if (ec == 6u) {          // critical edge
          const int lo = h + S.nb(k);
          const int eid = k < 7 ? 7 * h + k : 7 * lo + (k - 7);
          const int32_t f = A.edge_pos_of[eid];
          if (f < 0 && int64_t(-1 - f) < A.nedges) continue;  // dies in dimension 0
          if (f < 0 || int64_t(f) >= A.nedges || A.edge_ids[f] != eid) {
            atomicOr(A.err, 16);
            continue;
          }
          ++toggles;
          if (!toggle_row(Rows, rstride, &rl, rcap, uint32_t(f), &moved)) {
            ok = false;
            break;
          }
          continue;
        }
        const uint32_t stp = c_st.edge_step[k][ec];
        if (!(stp >> 31)) {
          atomicOr(A.err, 128);
          ok = false;
          break;
        }
        const int k2 = int(stp & 15u);
        ++expands;
        const uint32_t rn = N.get(k2);
        M ^= 1u << k2;  // the edge (h, n2)
        Rk[int64_t(k2) * rstride] = rn;
        if (ro > rn) {
          ok = H.push((uint64_t(ro) << 32) | rn, (uint32_t(h + S.nb(k)) << 4) | ((stp >> 4) & 15u));
        } else {
          ok = H.push((uint64_t(rn) << 32) | ro, (uint32_t(h + S.nb(k2)) << 4) | ((stp >> 8) & 15u));
        }
      }
    }
  } else
  while (ok && H.size() > 0) {
    if (++steps > A.max_steps) {
      ok = false;
      break;
    }
    maxlen = max(maxlen, H.size());
    uint64_t key;
    uint32_t ref;
    H.pop(&key, &ref);
    int copies = 1;
    while (H.size() > 0 && H.top_key() == key) {
      uint64_t k2;
      uint32_t r2;
      H.pop(&k2, &r2);
      ++copies;
    }
    if ((copies & 1) == 0) continue;  // cancels mod 2
    const int h = int(ref >> 4), k = int(ref & 15u);
    if (h != code_v) {
      code_v = h;
      ++groups;
      code_h = N.start(h);
    }
    if (H.size() > 0) {
      const int nh = int(H.top_ref() >> 4);
      if (nh != h) N.hint(nh);
    }
    const uint32_t ec = edge_code(code_h, k);
    if (ec == 7u) continue;  // paired with its vertex: the path ends
    if (ec == 6u) {          // critical edge
      const int lo = h + S.nb(k);
      const int eid = k < 7 ? 7 * h + k : 7 * lo + (k - 7);
      // its position among the critical edges, or -1 - position if it dies
      // in dimension 0 (dropped)
      const int32_t f = A.edge_pos_of[eid];
      if (f < 0 && int64_t(-1 - f) < A.nedges) continue;
      if (f < 0 || int64_t(f) >= A.nedges || A.edge_ids[f] != eid) {
        if (lead) atomicOr(A.err, 16);
        continue;
      }
      const uint32_t row = uint32_t(f);
      ++toggles;
      if (!toggle_row(Rows, rstride, &rl, rcap, row, &moved)) {
        ok = false;
        break;
      }
      continue;
    }
    // paired with the ec-th star triangle (h, o, n2) containing the edge
    const uint32_t stp = c_st.edge_step[k][ec];
    if (!(stp >> 31)) {
      if (lead) atomicOr(A.err, 128);
      ok = false;
      break;
    }
    const int k2 = int(stp & 15u);
    ++expands;
    const uint32_t rh = uint32_t(key >> 32), ro = uint32_t(key);
    const uint32_t rn = N.get(k2);
    // edges (h, n2) and (o, n2)
    ok = H.push((uint64_t(rh) << 32) | rn, (uint32_t(h) << 4) | uint32_t(k2));
    if (ok) {
      const int o = h + S.nb(k);
      if (ro > rn) {
        ok = H.push((uint64_t(ro) << 32) | rn, (uint32_t(o) << 4) | ((stp >> 4) & 15u));
      } else {
        const int n2 = h + S.nb(k2);
        ok = H.push((uint64_t(rn) << 32) | ro, (uint32_t(n2) << 4) | ((stp >> 8) & 15u));
      }
    }
  }
  if (!lead) return;  // the rest is done once per column
  if (A.stats) {  // expansion statistics (diagnostics)
    atomicAdd(&A.stats[0], (unsigned long long)steps);
    atomicMax(&A.stats[1], (unsigned long long)steps);
    atomicMax(&A.stats[2], (unsigned long long)maxlen);
    if (steps > 1000) atomicAdd(&A.stats[3], 1ull);
    if (!ok) atomicAdd(&A.stats[4], 1ull);
    atomicAdd(&A.stats[5 + min(31 - __clz(steps | 1), 20)], 1ull);
    // largest heap: <= 8, 16, 32, 64, 128, more
    atomicAdd(&A.stats[26 + min(max(31 - __clz(max(maxlen - 1, 1)) - 2, 0), 5)], 1ull);
    atomicAdd(&A.stats[32], (unsigned long long)toggles);
    atomicAdd(&A.stats[33], (unsigned long long)moved);
    atomicAdd(&A.stats[34], (unsigned long long)groups);
    atomicAdd(&A.stats[35], (unsigned long long)expands);
    if (steps > 2000) {  // the long columns
      atomicAdd(&A.stats[36], (unsigned long long)steps);
      atomicAdd(&A.stats[37], (unsigned long long)toggles);
      atomicAdd(&A.stats[38], (unsigned long long)moved);
      atomicAdd(&A.stats[39], (unsigned long long)groups);
    }
  }
  if (!ok) {
    A.retry[atomicAdd(A.nretry, 1u)] = c;
    return;
  }
  if (rl == 0) {
    atomicOr(A.err, 32);  // a negative triangle must have a non-empty boundary
    A.col_desc[c] = 0;
    return;
  }
  const unsigned long long at = atomicAdd(A.pool.top, (unsigned long long)rl);
  if ((int64_t)(at + rl) > A.pool.cap) {
    atomicOr(A.pool_full, 1);  // retried after growing the pool
    A.retry[atomicAdd(A.nretry, 1u)] = c;
    return;
  }
  for (int i = 0; i < rl; ++i) A.pool.data[at + i] = Rows[int64_t(rl - 1 - i) * rstride];
  A.col_desc[c] = (uint64_t(at) << 24) | uint64_t(rl);
}

// First pass over every column: one lane per column, heap (16 entries) and
// rows (16) in LDS, interleaved by lane; a column that needs more is retried.
// (The columns are taken in key order: sorting them by grid position cut
// this kernel's HBM reads by 38 % but made it 24 % slower.)
constexpr int kLaneHeap = 16, kLaneRows = 16, kLaneThreads = 256;
template <class Geo>
__global__ void __launch_bounds__(kLaneThreads)
k_d1_boundary_lanes(BoundaryArgs<Geo> A, const uint32_t* __restrict__ todo, int64_t ntodo) {
  __shared__ uint64_t s_key[kLaneHeap * kLaneThreads];
  __shared__ uint32_t s_ref[kLaneHeap * kLaneThreads];
  __shared__ uint32_t s_rows[kLaneRows * kLaneThreads];
  __shared__ uint32_t s_rk[14 * kLaneThreads];  // ranks of a vertex group's members
  LaneHeap H;
  H.key = s_key + threadIdx.x;
  H.ref = s_ref + threadIdx.x;
  H.stride = kLaneThreads;
  H.cap = kLaneHeap;
  for (int64_t w = int64_t(blockIdx.x) * kLaneThreads + threadIdx.x; w < ntodo;
       w += int64_t(gridDim.x) * kLaneThreads)
    // every column, the last first: the columns of the highest triangles
    // have the longest expansions, and the blocks are dispatched in order
    boundary_column<false, LaneHeap, Geo, true>(A, todo ? todo[w] : uint32_t(ntodo - 1 - w), H,
                                                s_rows + threadIdx.x, kLaneThreads, kLaneRows,
                                                s_rk + threadIdx.x);
}

constexpr int kWaveRegs = 4, kWaveRegs2 = 16;  // entries a lane in the two wave passes
// Long columns: one column per wave, the queue in the wave's registers (up to
// 64 R edges: 256, and 1024 for the columns that outgrow that), rows in LDS;
// the pops are sequential, each a few cross-lane moves, with the next vertex
// group's code and neighbour ranks loaded ahead.
constexpr int kWaveRows = 1024;
template <class Geo, int R>
__global__ void __launch_bounds__(64)
k_d1_boundary_wave(BoundaryArgs<Geo> A, const uint32_t* __restrict__ todo, int64_t ntodo,
                   unsigned int* __restrict__ next) {
  __shared__ uint32_t s_rows[kWaveRows];
  WaveListR<R> H;
  H.cap = R == kWaveRegs ? A.wave_cap : A.wave2_cap;
  for (;;) {  // columns are taken from a shared counter, so long ones do not queue up
    unsigned int w = 0;
    if (threadIdx.x == 0) w = atomicAdd(next, 1u);
    w = lane_value(w, 0);
    if (int64_t(w) >= ntodo) break;
    boundary_column<true>(A, todo[w], H, s_rows, 1, kWaveRows);
  }
}

// Columns whose queue outgrows the wave's registers: one column per
// workgroup of one wave, heap and rows in LDS, expanded by the first lane.
constexpr int kLdsHeap = 2048, kLdsRows = 1024;
template <class Geo>
__global__ void __launch_bounds__(64)
k_d1_boundary_lds(BoundaryArgs<Geo> A, const uint32_t* __restrict__ todo, int64_t ntodo) {
  __shared__ uint64_t s_key[kLdsHeap];
  __shared__ uint32_t s_ref[kLdsHeap];
  __shared__ uint32_t s_rows[kLdsRows];
  if (threadIdx.x != 0) return;
  LaneHeap H;
  H.key = s_key;
  H.ref = s_ref;
  H.stride = 1;
  H.cap = kLdsHeap;
  for (int64_t w = blockIdx.x; w < ntodo; w += gridDim.x)
    boundary_column<false>(A, todo[w], H, s_rows, 1, kLdsRows);
}

// Parallel Z2 reduction.  owner[p] is the lowest column whose current pivot
// is p (never reset: a column only changes while it does not own its pivot).
// A round: every active column claims its pivot (atomicMin); an owner that
// loses its pivot to a lower column becomes active again; then every active
// column that does not own its pivot adds the owner's column (a column of
// lower index, so the result is a valid left-to-right reduction whose pivots
// are those of the standard algorithm).

__device__ __forceinline__ void d1_claim_one(uint32_t c, const uint64_t* __restrict__ col_desc,
                                             const uint32_t* __restrict__ pool,
                                             unsigned int* __restrict__ owner,
                                             unsigned int* __restrict__ mark, unsigned int round,
                                             uint32_t* __restrict__ list,
                                             unsigned int* __restrict__ nlist) {
  const uint64_t d = col_desc[c];
  if ((d & 0xFFFFFFu) == 0) return;
  const uint32_t piv = pool[d >> 24];
  const unsigned int old = atomicMin(&owner[piv], c);
  if (old != 0xFFFFFFFFu && old > c) {
    // `old` lost its pivot: it joins this round's active set once
    if (atomicExch(&mark[old], round) != round) list[atomicAdd(nlist, 1u)] = old;
  }
}

// Every member of the active list carries the current round in mark[].
// Device counters: cnt[0] = size of the current list (grows while owners
// are displaced), cnt[1] = size of the next list, cnt[2] = size of the
// current list when the round began.
// cnt[3]: long columns deferred to the workgroup kernel this round;
// cnt[4]: the lowest active column (every column below it is final);
// cnt[5]: columns deferred from the lane kernel to the wave kernel.
__global__ void k_d1_round_begin(unsigned int* __restrict__ cnt) {
  cnt[2] = cnt[0];
  cnt[1] = 0;
  cnt[3] = 0;
  cnt[4] = 0xFFFFFFFFu;
  cnt[5] = 0;
}

// end of a round: the next list becomes current, the round advances and the
// next round begins
__global__ void k_d1_round_next(unsigned int* __restrict__ cnt, unsigned int* __restrict__ round_ptr) {
  cnt[0] = cnt[1];
  *round_ptr += 1;
  cnt[2] = cnt[0];
  cnt[1] = 0;
  cnt[3] = 0;
  cnt[4] = 0xFFFFFFFFu;
  cnt[5] = 0;
}

// pdesc[p] = the column of p's owner (after the claims of a round, the owner
// of every claimed pivot keeps its column for the rest of the round), so that
// a reduction step loads the owner and its column at once.  An owner column of
// at most kInlineRows + 1 rows also has its rows after the pivot in
// prow[2p .. 2p + 1] (zeros after the last), so that the wave reduction reads
// them with the descriptor instead of after it.
constexpr uint32_t kInlineRows = 8;
__global__ void k_d1_publish(const uint64_t* __restrict__ col_desc, const uint32_t* __restrict__ pool,
                             const unsigned int* __restrict__ owner, const uint32_t* __restrict__ list,
                             const unsigned int* __restrict__ cnt, int64_t nall,
                             uint64_t* __restrict__ pdesc, uint4* __restrict__ prow) {
  const int64_t n = list ? int64_t(cnt[2]) : nall;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t c = list ? list[j] : uint32_t(j);
    const uint64_t d = col_desc[c];
    const uint32_t len = uint32_t(d & 0xFFFFFFu);
    if (len == 0) continue;
    const uint64_t off = d >> 24;
    const uint32_t piv = pool[off];
    if (owner[piv] != c) continue;
    pdesc[piv] = d;
    if (len <= kInlineRows + 1) {
      uint32_t r[kInlineRows];
#pragma unroll
      for (uint32_t i = 0; i < kInlineRows; ++i) r[i] = 1 + i < len ? pool[off + 1 + i] : 0u;
      prow[2 * int64_t(piv)] = make_uint4(r[0], r[1], r[2], r[3]);
      prow[2 * int64_t(piv) + 1] = make_uint4(r[4], r[5], r[6], r[7]);
    }
  }
}

__global__ void k_d1_claim(const uint64_t* __restrict__ col_desc, const uint32_t* __restrict__ pool,
                           unsigned int* __restrict__ owner, unsigned int* __restrict__ mark,
                           const unsigned int* __restrict__ round_ptr, uint32_t* __restrict__ list,
                           unsigned int* __restrict__ cnt) {
  const unsigned int n0 = cnt[2];
  const unsigned int round = *round_ptr;
  uint32_t lowest = 0xFFFFFFFFu;
  for (unsigned int j = blockIdx.x * blockDim.x + threadIdx.x; j < n0; j += gridDim.x * blockDim.x) {
    const uint32_t c = list[j];
    lowest = min(lowest, c);
    d1_claim_one(c, col_desc, pool, owner, mark, round, list, &cnt[0]);
  }
  for (int sh = 32; sh >= 1; sh >>= 1) lowest = min(lowest, uint32_t(__shfl_xor(int(lowest), sh, 64)));
  if ((threadIdx.x & 63u) == 0 && lowest != 0xFFFFFFFFu) atomicMin(&cnt[4], lowest);
}


// ---- wave-cooperative reduction of one column ----------------------------
// The working column stays in LDS while it is reduced against a chain of
// owner columns; each owner column is loaded by the whole wave and the
// symmetric difference of two descending lists is formed in parallel: an
// element x of list A kept in the result goes to slot
//   2 * (#kept elements of A before x) - (index of x in A) + (#elements of B greater than x).
constexpr int kWaveCap = 512;    // longest column handled in LDS
constexpr int kRedWaves = 4;     // waves per block of the cooperative kernels

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of elements of the descending list L[0..n) that are greater than x
__device__ __forceinline__ uint32_t count_greater(const uint32_t* L, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (L[mid] > x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// out = A xor B (both descending, unique); returns the length
__device__ uint32_t wave_xor(const uint32_t* A, uint32_t a, const uint32_t* B, uint32_t b,
                             uint32_t* out) {
  const unsigned lane = lane_id();
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t keptA = 0, keptB = 0;
  for (uint32_t base = 0; base < a; base += 64) {
    const uint32_t i = base + lane;
    bool keep = false;
    uint32_t r = 0;
    if (i < a) {
      r = count_greater(B, b, A[i]);
      keep = !(r < b && B[r] == A[i]);
    }
    const uint64_t m = __ballot(keep);
    const uint32_t pre = keptA + __popcll(m & lt);
    if (keep) out[2 * pre - i + r] = A[i];
    keptA += __popcll(m);
  }
  for (uint32_t base = 0; base < b; base += 64) {
    const uint32_t j = base + lane;
    bool keep = false;
    uint32_t r = 0;
    if (j < b) {
      r = count_greater(A, a, B[j]);
      keep = !(r < a && A[r] == B[j]);
    }
    const uint64_t m = __ballot(keep);
    const uint32_t pre = keptB + __popcll(m & lt);
    if (keep) out[2 * pre - j + r] = B[j];
    keptB += __popcll(m);
  }
  wave_sync();
  return keptA + keptB;
}

// Wave reduction of column c: returns 0 if c owns its pivot, 1 if it must be
// reduced again next round, 2 if the pool is full (column unchanged), -1 if
// the column or its owner is too long for LDS (the caller hands it to the
// workgroup kernel).
__device__ int d1_reduce_wave(uint32_t c, uint64_t* __restrict__ col_desc, uint32_t* __restrict__ pool,
                              const ColPool& pc, const unsigned int* __restrict__ owner,
                              const uint64_t* __restrict__ pdesc, const uint4* __restrict__ prow,
                              int* __restrict__ err, uint32_t fin, uint32_t* bufA, uint32_t* bufB,
                              uint32_t* bufO, unsigned long long* __restrict__ stats) {
  const unsigned lane = lane_id();
  const uint64_t d = col_desc[c];
  uint32_t len = uint32_t(d & 0xFFFFFFu);
  if (len == 0) return 0;
  if (len > kWaveCap) return -1;
  const uint64_t off = d >> 24;
  for (uint32_t i = lane; i < len; i += 64) bufA[i] = pool[off + i];
  wave_sync();
  bool changed = false;
  int result = 1;
  int steps_done = 0;
  uint32_t* cur = bufA;
  uint32_t* nxt = bufO;
  // the owner of the current pivot and its column; after the first step they
  // are loaded during the previous addition (the next pivot, the largest
  // row left after cancelling, is known from the two columns' heads)
  unsigned int o = owner[cur[0]];
  uint64_t od = pdesc[cur[0]];
  uint4 or0 = prow[2 * int64_t(cur[0])], or1 = prow[2 * int64_t(cur[0]) + 1];
  for (int steps = 0;; ++steps) {
    if (steps > (1 << 20)) {  // pivots strictly decrease: cannot happen
      if (lane == 0) atomicOr(err, 512);
      break;
    }
    if (o == c) {
      result = 0;
      break;
    }
    if (o > c) break;  // unowned or owned by a later column: claim next round
    const uint32_t olen = uint32_t(od & 0xFFFFFFu);
    if (olen > kWaveCap || len + olen > 2 * kWaveCap) {
      if (!changed) return -1;
      break;  // write back what we have; the next round hands it on
    }
    const uint64_t ooff = od >> 24;
    if (olen <= kInlineRows + 1) {  // the rows came with the descriptor
      const uint32_t e[kInlineRows] = {or0.x, or0.y, or0.z, or0.w, or1.x, or1.y, or1.z, or1.w};
      uint32_t v = cur[0];  // the owner's pivot is the current pivot
#pragma unroll
      for (uint32_t t = 0; t < kInlineRows; ++t)
        if (lane == t + 1) v = e[t];
      if (lane < olen) bufB[lane] = v;
    } else {
      for (uint32_t i = lane; i < olen; i += 64) bufB[i] = pool[ooff + i];
    }
    wave_sync();
    const unsigned int o_step = o;  // the owner added in this step
    uint32_t hi = 1, hj = 1;  // both heads are the pivot
    while (hi < len && hj < olen && cur[hi] == bufB[hj]) {
      ++hi;
      ++hj;
    }
    if (hi < len || hj < olen) {
      const uint32_t np = hi < len && (hj >= olen || cur[hi] > bufB[hj]) ? cur[hi] : bufB[hj];
      o = owner[np];
      od = pdesc[np];
      or0 = prow[2 * int64_t(np)];
      or1 = prow[2 * int64_t(np) + 1];
    }
    const uint32_t w = wave_xor(cur, len, bufB, olen, nxt);
    changed = true;
    ++steps_done;
    if (w == 0) {
      if (lane == 0) atomicOr(err, 64);
      len = 0;
      break;
    }
    uint32_t* t = cur;
    cur = nxt;
    nxt = t;
    len = w;
    if (o_step >= fin || len > kWaveCap) break;  // owner not final: one step per round
  }
  if (stats && lane == 0) {  // diagnostics: columns, additions, longest chain
    atomicAdd(&stats[0], 1ull);
    atomicAdd(&stats[1], (unsigned long long)steps_done);
    atomicMax(&stats[2], (unsigned long long)steps_done);
  }
  if (!changed) return result;
  unsigned long long at = 0;
  if (lane == 0) at = atomicAdd(pc.top, (unsigned long long)len);
  at = __shfl(at, 0, 64);
  if ((int64_t)(at + len) > pc.cap) return 2;  // column unchanged; retried after growth
  for (uint32_t i = lane; i < len; i += 64) pool[at + i] = cur[i];
  __threadfence();
  if (lane == 0) col_desc[c] = (uint64_t(at) << 24) | uint64_t(len);
  return result;
}

// ---- workgroup reduction of a long column -------------------------------
constexpr int kLongThreads = 1024;

// Exclusive prefix sums over the workgroup of two 0/1 flags packed as
// fa | fb << 16 (a workgroup holds at most 1024 lanes, so each sum fits in
// 16 bits); *total receives both sums packed the same way.  The per-wave
// totals are scanned by the first wave with shuffles.
__device__ __forceinline__ uint32_t block_scan2(uint32_t v, uint32_t* s_wave, uint32_t* total) {
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const unsigned nw = blockDim.x / 64;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint64_t ma = __ballot(v & 1u), mb = __ballot((v >> 16) & 1u);
  const uint32_t in_wave = uint32_t(__popcll(ma & lt)) | (uint32_t(__popcll(mb & lt)) << 16);
  if (lane == 0) s_wave[wave] = uint32_t(__popcll(ma)) | (uint32_t(__popcll(mb)) << 16);
  __syncthreads();
  if (wave == 0) {
    const uint32_t c = lane < nw ? s_wave[lane] : 0u;
    uint32_t x = c;  // inclusive scan; packed halves never carry (sums <= 1024)
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = uint32_t(__shfl_up(int(x), d, 64));
      if (int(lane) >= d) x += y;
    }
    if (lane < nw) s_wave[lane] = x - c;
    if (lane == nw - 1) s_wave[nw] = x;
  }
  __syncthreads();
  const uint32_t r = s_wave[wave] + in_wave;
  *total = s_wave[nw];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint32_t count_greater_g(const uint32_t* __restrict__ L, uint32_t n,
                                                    uint32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (L[mid] > x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Symmetric difference of the descending lists A (a) and B (b) into out,
// by the whole workgroup; returns the result length.
__device__ uint32_t block_xor(const uint32_t* A, uint32_t a, const uint32_t* B, uint32_t b,
                              uint32_t* out, uint32_t* s_wave) {
  // one pass: lane t of chunk k takes A[k * 1024 + t] and B[k * 1024 + t]; an
  // element kept from A lands at 2 * (kept A before it) - i + (B elements
  // greater than it), and symmetrically for B
  uint32_t keptA = 0, keptB = 0, tot;
  const uint32_t n = a > b ? a : b;
  for (uint32_t base = 0; base < n; base += kLongThreads) {
    const uint32_t i = base + threadIdx.x;
    uint32_t ka = 0, kb = 0, ra = 0, rb = 0, xa = 0, xb = 0;
    if (i < a) {
      xa = A[i];
      ra = count_greater_g(B, b, xa);
      ka = !(ra < b && B[ra] == xa);
    }
    if (i < b) {
      xb = B[i];
      rb = count_greater_g(A, a, xb);
      kb = !(rb < a && A[rb] == xb);
    }
    const uint32_t pre = block_scan2(ka | (kb << 16), s_wave, &tot);
    if (ka) out[2 * (keptA + (pre & 0xFFFFu)) - i + ra] = xa;
    if (kb) out[2 * (keptB + (pre >> 16)) - i + rb] = xb;
    keptA += tot & 0xFFFFu;
    keptB += tot >> 16;
  }
  __syncthreads();
  return keptA + keptB;
}

// Exclusive prefix sum over the workgroup of small per-thread counts;
// *total receives the sum.
__device__ __forceinline__ uint32_t block_scan_counts(uint32_t v, uint32_t* s_wave,
                                                      uint32_t* total) {
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const unsigned nw = blockDim.x / 64;
  uint32_t x = v;  // inclusive scan within the wave
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = uint32_t(__shfl_up(int(x), d, 64));
    if (int(lane) >= d) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  if (wave == 0) {
    const uint32_t c = lane < nw ? s_wave[lane] : 0u;
    uint32_t z = c;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = uint32_t(__shfl_up(int(z), d, 64));
      if (int(lane) >= d) z += y;
    }
    if (lane < nw) s_wave[lane] = z - c;
    if (lane == nw - 1) s_wave[nw] = z;
  }
  __syncthreads();
  const uint32_t r = s_wave[wave] + x - v;
  *total = s_wave[nw];
  __syncthreads();
  return r;
}

// Symmetric difference of the descending lists A (a) and B (b), both in LDS,
// by the whole workgroup: a merge-path merge into tmp (thread t writes the
// merged positions [t K, (t + 1) K), K = ceil((a + b) / threads), starting
// from the split found by one binary search on its diagonal; on equal values
// A's comes first), then the equal pairs, which are neighbours in the merged
// list, are dropped while the rest is compacted into out.  Two passes over
// short per-thread runs instead of one binary search per element.
__device__ uint32_t block_xor_merge(const uint32_t* A, uint32_t a, const uint32_t* B, uint32_t b,
                                    uint32_t* tmp, uint32_t* out, uint32_t* s_wave) {
  const uint32_t total = a + b;
  const uint32_t K = (total + kLongThreads - 1) / kLongThreads;
  const uint32_t d0 = min(threadIdx.x * K, total), d1 = min(d0 + K, total);
  // i = number of A elements among the first d0 merged ones: the first i in
  // [max(0, d0 - b), min(d0, a)] with A[i] after B[d0 - 1 - i]
  uint32_t lo = d0 > b ? d0 - b : 0u, hi = d0 < a ? d0 : a;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (A[mid] >= B[d0 - 1 - mid]) lo = mid + 1;  // A[mid] comes first
    else hi = mid;
  }
  uint32_t i = lo, j = d0 - lo;
  for (uint32_t p = d0; p < d1; ++p) {
    if (i < a && (j >= b || A[i] >= B[j])) tmp[p] = A[i++];
    else tmp[p] = B[j++];
  }
  __syncthreads();
  uint64_t keep = 0;  // K <= kLongCap / kLongThreads <= 64
  uint32_t cnt = 0;
  for (uint32_t p = d0; p < d1; ++p) {
    const uint32_t x = tmp[p];
    const bool gone = (p + 1 < total && tmp[p + 1] == x) || (p > 0 && tmp[p - 1] == x);
    if (!gone) {
      keep |= 1ull << (p - d0);
      ++cnt;
    }
  }
  uint32_t kept;
  uint32_t at = block_scan_counts(cnt, s_wave, &kept);
  for (uint32_t p = d0; p < d1; ++p)
    if ((keep >> (p - d0)) & 1ull) out[at++] = tmp[p];
  __syncthreads();
  return kept;
}

// Reduce phase for long columns, one workgroup per column.  The working
// column stays in LDS across the additions of a round (chained through
// final owners) and is written back once; a column or owner too long for
// the LDS buffers is reduced in global memory instead.
constexpr uint32_t kLongCap = 12288;
__global__ void __launch_bounds__(kLongThreads)
k_d1_reduce_long(uint64_t* __restrict__ col_desc, uint32_t* __restrict__ pool, ColPool pc,
                 const unsigned int* __restrict__ owner, const uint64_t* __restrict__ pdesc,
                 const uint4* __restrict__ prow, unsigned int* __restrict__ mark,
                 unsigned int* __restrict__ round_ptr, const uint32_t* __restrict__ long_list,
                 uint32_t* __restrict__ next, unsigned int* __restrict__ cnt, int* __restrict__ err,
                 int* __restrict__ pool_full, unsigned long long* __restrict__ stats) {
  __shared__ uint32_t s_col[2][kLongCap];
  __shared__ uint32_t s_own[kLongCap];
  __shared__ uint32_t s_wave[kLongThreads / 64 + 1];
  __shared__ uint64_t s_off, s_ooff;
  __shared__ unsigned long long s_at;
  __shared__ uint32_t s_len, s_olen;
  __shared__ int s_state;  // -1 continue, 0 owner, 1 next round, 2 pool full, 3 stop (error)
  __shared__ int s_lds;    // the working column lives in s_col[cur]
  __shared__ int s_spill;  // it must move to global memory before the next addition
  // the owner of the next pivot and its column, loaded during the addition
  // before (the next pivot is known from the two columns' heads)
  __shared__ int s_pf;
  __shared__ unsigned int s_po;
  __shared__ uint64_t s_pod;
  // the inline rows of the current owner, and those loaded with the next one
  __shared__ uint4 s_rec[2], s_prf[2];
  // a short owner's rows: their places in the working column, and hits
  __shared__ uint32_t s_fpos[kInlineRows], s_fhit[kInlineRows];
  const unsigned int nlong = cnt[3];
  const unsigned int round = *round_ptr;
  const uint32_t fin = cnt[4];  // owners below it are final
  for (unsigned int b = blockIdx.x; b < nlong; b += gridDim.x) {
    const uint32_t c = long_list[b];
    if (threadIdx.x == 0) {
      const uint64_t d = col_desc[c];
      s_len = uint32_t(d & 0xFFFFFFu);
      s_off = d >> 24;
      s_lds = s_len <= kLongCap ? 1 : 0;
      s_state = -1;
      s_pf = 0;
    }
    __syncthreads();
    int cur = 0, nsteps = 0;
    uint64_t tph[4] = {0, 0, 0, 0};  // diagnostics: decision, owner load, merge, update
    uint64_t tmark = wall_clock64();
    bool dirty = false;  // the LDS column is newer than col_desc[c]
    if (s_lds)
      for (uint32_t i = threadIdx.x; i < s_len; i += kLongThreads) s_col[0][i] = pool[s_off + i];
    __syncthreads();
    for (int steps = 0;; ++steps) {
      // the next owner, loaded by thread 0 during this addition
      unsigned int po = 0;
      uint64_t pod = 0;
      uint4 pr0 = make_uint4(0, 0, 0, 0), pr1 = make_uint4(0, 0, 0, 0);
      bool pf = false;
      // the next pivot from the heads of the working column and the owner
      // (both heads are the pivot); its owner's loads are issued at once
      auto prefetch_next = [&](const uint32_t* X, auto own) {
        uint32_t hi = 1, hj = 1;
        while (hi < s_len && hj < s_olen && X[hi] == own(hj)) {
          ++hi;
          ++hj;
        }
        if (hi < s_len || hj < s_olen) {
          const uint32_t np = hi < s_len && (hj >= s_olen || X[hi] > own(hj)) ? X[hi] : own(hj);
          po = owner[np];
          pod = pdesc[np];
          pr0 = prow[2 * int64_t(np)];
          pr1 = prow[2 * int64_t(np) + 1];
          pf = true;
        }
      };
      if (threadIdx.x == 0) {
        s_state = -1;
        s_spill = 0;
        if (s_len == 0 || steps > (1 << 22)) {
          s_state = 3;
          atomicOr(err, 1024);
        } else {
          unsigned int o;
          uint64_t od;  // the owner's column, loaded with the owner
          if (s_pf) {
            o = s_po;
            od = s_pod;
            s_rec[0] = s_prf[0];
            s_rec[1] = s_prf[1];
          } else {
            const uint32_t piv = s_lds ? s_col[cur][0] : pool[s_off];
            o = owner[piv];
            od = pdesc[piv];
            s_rec[0] = prow[2 * int64_t(piv)];
            s_rec[1] = prow[2 * int64_t(piv) + 1];
          }
          s_pf = 0;
          if (o == c) {
            s_state = 0;
          } else if (o > c || (steps > 0 && o >= fin)) {
            s_state = 1;  // unowned, owned later, or owner not final: next round
          } else {
            s_olen = uint32_t(od & 0xFFFFFFu);
            s_ooff = od >> 24;
            if (s_lds && (s_olen > kLongCap || s_len + s_olen > kLongCap)) s_spill = 1;
            if (s_lds && !s_spill && s_olen <= kInlineRows + 1) {
              // a short owner: its rows are at hand, so the next owner's
              // loads are issued before the barrier
              const uint32_t* rec = reinterpret_cast<const uint32_t*>(s_rec);
              prefetch_next(s_col[cur], [&](uint32_t j) { return rec[j - 1]; });
            }
          }
        }
      }
      __syncthreads();
      if (stats) {
        const uint64_t t = wall_clock64();
        tph[0] += t - tmark;
        tmark = t;
      }
      if (s_state >= 0) break;
      ++nsteps;
      if (s_spill) {
        if (dirty) {  // write the LDS column into the pool first
          if (threadIdx.x == 0) {
            s_at = atomicAdd(pc.top, (unsigned long long)s_len);
            if ((int64_t)(s_at + s_len) > pc.cap) s_state = 2;  // this round's progress is dropped
          }
          __syncthreads();
          if (s_state == 2) break;
          for (uint32_t i = threadIdx.x; i < s_len; i += kLongThreads) pool[s_at + i] = s_col[cur][i];
          __threadfence();
          __syncthreads();
          if (threadIdx.x == 0) {
            col_desc[c] = (uint64_t(s_at) << 24) | uint64_t(s_len);
            s_off = s_at;
          }
          dirty = false;
        }
        if (threadIdx.x == 0) s_lds = 0;
        __syncthreads();
      }
      if (s_lds) {
        // a short owner's rows after its pivot (the current pivot) came with
        // the descriptor and are read from s_rec; a longer one is loaded
        const bool short_owner = s_olen <= kInlineRows + 1;
        const uint32_t* rec = reinterpret_cast<const uint32_t*>(s_rec);
        if (!short_owner) {
          for (uint32_t i = threadIdx.x; i < s_olen; i += kLongThreads) s_own[i] = pool[s_ooff + i];
          __syncthreads();
        }
        if (stats) {
          const uint64_t t = wall_clock64();
          tph[1] += t - tmark;
          tmark = t;
        }
        if (threadIdx.x == 0 && !short_owner)  // (for a short owner: issued in the decision)
          prefetch_next(s_col[cur], [&](uint32_t j) { return s_own[j]; });
        uint32_t w;
        if (short_owner) {
          // A short owner (most of the additions of the long chains): each of
          // its rows below the pivot is searched in the working column (a hit
          // deletes that element, a miss inserts the row before position
          // pos), then every element moves once to its new place in
          // s_col[cur ^ 1], which becomes the working column: no merge and no
          // prefix scan.  Element i > 0 moves by -1 (the pivot) - (hits
          // before i) + (misses at or before i); the miss of row k lands at
          // pos - 1 - (hits before pos) + (misses of earlier rows).
          const uint32_t m = s_olen - 1, n = s_len;
          const uint32_t* Wc = s_col[cur];
          // wave k < m places row k: a 64-way search (64 samples a level,
          // compared in one step, counted with a ballot) needs three
          // dependent LDS reads for the longest columns instead of fourteen
          const uint32_t wv = threadIdx.x >> 6, ln = threadIdx.x & 63u;
          if (wv < m) {
            const uint32_t v = rec[wv];
            uint32_t lo = 0, hi = n;  // the count of elements above v lies in [lo, hi]
            while (hi - lo > 64) {
              const uint32_t span = hi - lo;
              const uint32_t at = lo + uint32_t((uint64_t(ln + 1) * span) / 65);
              const int c = __popcll(__ballot(Wc[at] > v));  // samples above v
              const uint32_t lo2 = c == 0 ? lo : lo + uint32_t((uint64_t(c) * span) / 65) + 1;
              const uint32_t hi2 = c == 64 ? hi : lo + uint32_t((uint64_t(c + 1) * span) / 65);
              lo = lo2;
              hi = hi2;
            }
            const uint32_t pos = lo + uint32_t(__popcll(__ballot(ln < hi - lo && Wc[lo + ln] > v)));
            if (ln == 0) {
              s_fpos[wv] = pos;
              s_fhit[wv] = (pos < n && Wc[pos] == v) ? 1u : 0u;
            }
          }
          __syncthreads();
          uint32_t fp[kInlineRows], fh[kInlineRows], nh = 0;
#pragma unroll
          for (uint32_t k = 0; k < kInlineRows; ++k) {
            fp[k] = k < m ? s_fpos[k] : 0xFFFFFFFFu;
            fh[k] = k < m ? s_fhit[k] : 0u;
            nh += fh[k];
          }
          uint32_t* out = s_col[cur ^ 1];
          for (uint32_t i = threadIdx.x + 1; i < n; i += kLongThreads) {
            int shift = -1;
            bool del = false;
#pragma unroll
            for (uint32_t k = 0; k < kInlineRows; ++k) {
              if (k >= m) continue;
              if (fh[k]) {
                if (fp[k] < i) --shift;
                else if (fp[k] == i) del = true;
              } else if (fp[k] <= i) {
                ++shift;
              }
            }
            if (!del) out[int(i) + shift] = Wc[i];
          }
          if (threadIdx.x < m && !s_fhit[threadIdx.x]) {
            const uint32_t pk = s_fpos[threadIdx.x];
            int at = int(pk) - 1;
            for (uint32_t k = 0; k < m; ++k) {
              if (s_fhit[k] && s_fpos[k] < pk) --at;
              if (!s_fhit[k] && k < threadIdx.x) ++at;
            }
            out[at] = rec[threadIdx.x];
          }
          __syncthreads();
          cur ^= 1;
          w = n - 1 - nh + (m - nh);
        } else {
          // merged into s_col[cur ^ 1], compacted back into s_col[cur]
          w = block_xor_merge(s_col[cur], s_len, s_own, s_olen, s_col[cur ^ 1], s_col[cur], s_wave);
        }
        if (stats) {
          const uint64_t t = wall_clock64();
          tph[2] += t - tmark;
          tmark = t;
        }
        dirty = true;
        if (threadIdx.x == 0) {
          if (w == 0) atomicOr(err, 64);  // a negative column cannot vanish
          s_len = w;
          if (pf) {
            s_po = po;
            s_pod = pod;
            s_prf[0] = pr0;
            s_prf[1] = pr1;
            s_pf = 1;
          }
        }
        // no barrier here: only thread 0 wrote, and only thread 0 reads
        // before the barrier after the next decision
        if (stats) {
          const uint64_t t = wall_clock64();
          tph[3] += t - tmark;
          tmark = t;
        }
      } else {
        if (threadIdx.x == 0) {
          s_at = atomicAdd(pc.top, (unsigned long long)(s_len + s_olen));
          if ((int64_t)(s_at + s_len + s_olen) > pc.cap) s_state = 2;
        }
        __syncthreads();
        if (s_state == 2) break;
        const uint32_t w = block_xor(pool + s_off, s_len, pool + s_ooff, s_olen, pool + s_at, s_wave);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
          if (w == 0) atomicOr(err, 64);
          col_desc[c] = (uint64_t(s_at) << 24) | uint64_t(w);
          s_len = w;
          s_off = s_at;
        }
        __threadfence();
        __syncthreads();
      }
    }
    // write back the LDS column
    if (dirty && (s_state == 0 || s_state == 1)) {
      if (threadIdx.x == 0) {
        s_at = atomicAdd(pc.top, (unsigned long long)s_len);
        if ((int64_t)(s_at + s_len) > pc.cap) s_state = 2;  // progress dropped
      }
      __syncthreads();
      if (s_state != 2) {
        for (uint32_t i = threadIdx.x; i < s_len; i += kLongThreads) pool[s_at + i] = s_col[cur][i];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) col_desc[c] = (uint64_t(s_at) << 24) | uint64_t(s_len);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (stats) {
        atomicAdd(&stats[3], 1ull);
        atomicAdd(&stats[4], (unsigned long long)nsteps);
        atomicMax(&stats[5], (unsigned long long)nsteps);
        for (int q = 0; q < 4; ++q) atomicAdd(&stats[8 + q], (unsigned long long)tph[q]);
      }
      int st = s_state;
      if (st == 0 && dirty) st = 1;  // the pivot changed this round: claim it next round
      if (st == 2) atomicOr(pool_full, 1);
      if (st == 1 || st == 2) {
        mark[c] = round + 1;
        next[atomicAdd(&cnt[1], 1u)] = c;
      }
    }
    __syncthreads();
  }
}

// Reduce phase with one wave per active column.
// ---- lane reduction of short columns -------------------------------------
// Most columns are a few rows long: one lane per column, the working column,
// the next one and the owner's column in LDS (interleaved by lane).  Same
// steps and results as the wave form; a column (or owner) longer than
// kLaneCol is deferred to the wave kernel of the same round.
constexpr int kLaneCol = 16, kRedLanes = 128;

__device__ __forceinline__ void load_col(const uint32_t* __restrict__ src, uint32_t n, uint32_t* dst) {
  uint32_t v[kLaneCol];
#pragma unroll
  for (int i = 0; i < kLaneCol; ++i) v[i] = uint32_t(i) < n ? src[i] : 0u;
#pragma unroll
  for (int i = 0; i < kLaneCol; ++i)
    if (uint32_t(i) < n) dst[i * kRedLanes] = v[i];
}

// returns as d1_reduce_wave: 0 owner, 1 again next round, 2 pool full, -1 deferred
__device__ int d1_reduce_lane(uint32_t c, uint64_t* __restrict__ col_desc, uint32_t* __restrict__ pool,
                              const ColPool& pc, const unsigned int* __restrict__ owner,
                              const uint64_t* __restrict__ pdesc, const uint4* __restrict__ prow,
                              int* __restrict__ err, uint32_t fin,
                              uint32_t* cur, uint32_t* nxt, uint32_t* own, int* adds) {
  const uint64_t d = col_desc[c];
  uint32_t len = uint32_t(d & 0xFFFFFFu);
  *adds = 0;
  if (len == 0) return 0;
  if (len > uint32_t(kLaneCol)) return -1;
  load_col(pool + (d >> 24), len, cur);
  bool changed = false;
  int result = 1;
  for (;;) {
    const uint32_t piv = cur[0];
    const unsigned int o = owner[piv];
    const uint64_t od = pdesc[piv];
    const uint4 r0 = prow[2 * int64_t(piv)], r1 = prow[2 * int64_t(piv) + 1];  // with od
    if (o == c) {
      result = 0;
      break;
    }
    if (o > c) break;  // unowned or owned by a later column: claim next round
    const uint32_t olen = uint32_t(od & 0xFFFFFFu);
    if (olen > uint32_t(kLaneCol) || len + olen > uint32_t(2 * kLaneCol)) {
      if (!changed) return -1;
      break;  // write back what we have; the next round hands it on
    }
    if (olen <= kInlineRows + 1) {  // the rows came with the descriptor
      const uint32_t e[kInlineRows + 1] = {piv, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
      for (uint32_t i = 0; i <= kInlineRows; ++i)
        if (i < olen) own[i * kRedLanes] = e[i];
    } else {
      load_col(pool + (od >> 24), olen, own);
    }
    // symmetric difference of the two descending lists
    uint32_t i = 0, j = 0, w = 0;
    while (i < len && j < olen) {
      const uint32_t x = cur[i * kRedLanes], y = own[j * kRedLanes];
      if (x == y) {
        ++i;
        ++j;
      } else if (x > y) {
        nxt[(w++) * kRedLanes] = x;
        ++i;
      } else {
        nxt[(w++) * kRedLanes] = y;
        ++j;
      }
    }
    for (; i < len; ++i) nxt[(w++) * kRedLanes] = cur[i * kRedLanes];
    for (; j < olen; ++j) nxt[(w++) * kRedLanes] = own[j * kRedLanes];
    changed = true;
    ++*adds;
    if (w == 0) {
      atomicOr(err, 64);
      len = 0;
      break;
    }
    uint32_t* t = cur;
    cur = nxt;
    nxt = t;
    len = w;
    if (o >= fin || len > uint32_t(kLaneCol)) break;  // owner not final: one step per round
  }
  if (!changed) return result;
  const unsigned long long at = atomicAdd(pc.top, (unsigned long long)len);
  if ((int64_t)(at + len) > pc.cap) return 2;  // column unchanged; retried after growth
  for (uint32_t i = 0; i < len; ++i) pool[at + i] = cur[i * kRedLanes];
  __threadfence();
  col_desc[c] = (uint64_t(at) << 24) | uint64_t(len);
  return result;
}

// append v to list (counter *n) for the lanes whose flag is set, with one
// atomic per wave
__device__ __forceinline__ void wave_append(bool flag, uint32_t v, uint32_t* __restrict__ list,
                                            unsigned int* __restrict__ n) {
  const uint64_t m = __ballot(flag);
  if (m == 0) return;
  const unsigned lane = threadIdx.x & 63u;
  const int first = __ffsll((unsigned long long)m) - 1;
  unsigned int base = 0;
  if (int(lane) == first) base = atomicAdd(n, unsigned(__popcll(m)));
  base = __shfl(base, first);
  if (flag) list[base + __popcll(m & ((1ull << lane) - 1))] = v;
}

__global__ void __launch_bounds__(kRedLanes)
k_d1_reduce_lanes(uint64_t* __restrict__ col_desc, uint32_t* __restrict__ pool, ColPool pc,
                  const unsigned int* __restrict__ owner, const uint64_t* __restrict__ pdesc,
                  const uint4* __restrict__ prow,
                  unsigned int* __restrict__ mark, unsigned int* __restrict__ round_ptr,
                  const uint32_t* __restrict__ list, uint32_t* __restrict__ next,
                  unsigned int* __restrict__ cnt, int* __restrict__ err, int* __restrict__ pool_full,
                  uint32_t* __restrict__ wave_list, unsigned long long* __restrict__ stats) {
  __shared__ uint32_t s_buf[(5 * kLaneCol) * kRedLanes];
  uint32_t* cur = s_buf + threadIdx.x;
  uint32_t* nxt = cur + 2 * kLaneCol * kRedLanes;
  uint32_t* own = nxt + 2 * kLaneCol * kRedLanes;
  const unsigned int n1 = cnt[0];
  const uint32_t fin = cnt[4];  // owners below it are final
  const unsigned int round = *round_ptr;
  // every lane of a wave runs the same number of iterations (ballots below)
  const unsigned int stride = gridDim.x * kRedLanes;
  const unsigned int begin = blockIdx.x * kRedLanes + (threadIdx.x & ~63u);
  for (unsigned int jb = begin; jb < n1; jb += stride) {
    const unsigned int j = jb + (threadIdx.x & 63u);
    const bool live = j < n1;
    const uint32_t c = live ? list[j] : 0u;
    int adds = 0;
    const int r = live ? d1_reduce_lane(c, col_desc, pool, pc, owner, pdesc, prow, err, fin, cur, nxt, own,
                                        &adds)
                       : 0;
    if (r == 2) atomicOr(pool_full, 1);
    if (live && r > 0) mark[c] = round + 1;
    wave_append(live && r > 0, c, next, &cnt[1]);
    wave_append(live && r < 0, c, wave_list, &cnt[5]);
    if (stats) {
      const uint64_t m = __ballot(live && r >= 0);
      int a = adds;
      for (int sh = 32; sh >= 1; sh >>= 1) a += __shfl_xor(a, sh, 64);
      if ((threadIdx.x & 63u) == 0) {
        atomicAdd(&stats[6], (unsigned long long)__popcll(m));
        atomicAdd(&stats[7], (unsigned long long)a);
      }
    }
  }
}

__global__ void __launch_bounds__(64 * kRedWaves)
k_d1_reduce_wave(uint64_t* __restrict__ col_desc, uint32_t* __restrict__ pool, ColPool pc,
                 const unsigned int* __restrict__ owner, const uint64_t* __restrict__ pdesc,
                 const uint4* __restrict__ prow, unsigned int* __restrict__ mark,
                 unsigned int* __restrict__ round_ptr, const uint32_t* __restrict__ list,
                 uint32_t* __restrict__ next, unsigned int* __restrict__ cnt, int* __restrict__ err,
                 int* __restrict__ pool_full, uint32_t* __restrict__ long_list,
                 unsigned long long* __restrict__ stats) {
  __shared__ uint32_t s_buf[kRedWaves][3][2 * kWaveCap];
  const unsigned wave = threadIdx.x >> 6;
  const unsigned lane = lane_id();
  const unsigned int n1 = cnt[5];  // the columns the lane kernel deferred
  const uint32_t fin = cnt[4];  // owners below it are final
  const unsigned int round = *round_ptr;
  const unsigned gw = blockIdx.x * kRedWaves + wave;
  const unsigned nw = gridDim.x * kRedWaves;
  for (unsigned int j = gw; j < n1; j += nw) {
    const uint32_t c = list[j];
    int r = d1_reduce_wave(c, col_desc, pool, pc, owner, pdesc, prow, err, fin, s_buf[wave][0], s_buf[wave][1],
                           s_buf[wave][2], stats);
    if (r < 0) {  // too long for the wave: handled by a whole workgroup this round
      if (lane == 0) long_list[atomicAdd(&cnt[3], 1u)] = c;
      wave_sync();
      continue;
    }
    if (lane == 0) {
      if (r == 2) atomicOr(pool_full, 1);
      if (r != 0) {
        mark[c] = round + 1;
        next[atomicAdd(&cnt[1], 1u)] = c;
      }
    }
    wave_sync();
  }
}

__global__ void k_fill_u32(unsigned int* a, int64_t n, unsigned int v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_col_lengths(const uint64_t* __restrict__ col_desc, int64_t ncols,
                              uint32_t* __restrict__ lens) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < ncols) lens[c] = uint32_t(col_desc[c] & 0xFFFFFFu);
  if (c == ncols) lens[c] = 0;
}

__global__ void k_col_compact(uint64_t* __restrict__ col_desc, int64_t ncols,
                              const uint32_t* __restrict__ pool, const uint32_t* __restrict__ offs,
                              uint32_t* __restrict__ out) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const uint64_t d = col_desc[c];
  const uint32_t len = uint32_t(d & 0xFFFFFFu);
  const uint64_t from = d >> 24;
  const uint64_t to = offs[c];
  for (uint32_t i = 0; i < len; ++i) out[to + i] = pool[from + i];
  col_desc[c] = (to << 24) | uint64_t(len);
}

__global__ void k_set_u64(unsigned long long* a, uint64_t v) { *a = v; }

__global__ void k_fill_u64(uint64_t* a, int64_t n, uint64_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_u8(uint8_t* a, int64_t n, uint8_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// columns of D1 (triangles not paired in D2), in no particular order
__global__ void k_collect_cols(const uint8_t* __restrict__ tri_state, int64_t nt,
                               uint32_t* __restrict__ cols, unsigned int* __restrict__ ncols) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool take = i < nt && tri_state[i] == 1;
  const unsigned int at = block_append(take, ncols);
  if (take) cols[at] = uint32_t(i);
}

__global__ void k_d1_pairs(const uint64_t* __restrict__ col_desc, int64_t ncols,
                           const uint32_t* __restrict__ cols, const uint32_t* __restrict__ pool,
                           const int32_t* __restrict__ edge_ids, const uint64_t* __restrict__ edge_keys,
                           const int32_t* __restrict__ tri_ids, const uint64_t* __restrict__ tri_keys,
                           PairOut po) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t d = 0;
  if (c < ncols) d = col_desc[c];
  const bool take = c < ncols && (d & 0xFFFFFFu) != 0;  // an empty column pairs nothing
  const unsigned long long p = block_append(take, po.count);
  if (!take) return;
  const uint32_t row = pool[d >> 24];
  const uint32_t ti = cols[c];
  if ((int64_t)p < po.cap) {
    po.dim[p] = 1;
    po.birth[p] = edge_ids[row];
    po.death[p] = tri_ids[ti];
    po.bkey[p] = edge_keys[row];
    po.dkey[p] = tri_keys[ti];
  }
}

// ======================================================================
// K8: diagram
// ======================================================================

// Lowest and highest rank of every field of a batch (the essential class of
// a field is born at its lowest vertex and paired with its highest).  A lane
// scans kAppendPer vertices (stride 256) and flushes its running extremes
// when the field changes; a wave whose lanes end in one field reduces them
// and issues one atomic pair.
__global__ void __launch_bounds__(256)
k_field_extrema(const int32_t* __restrict__ rank, GeoBatch G, unsigned int* __restrict__ fmin,
                unsigned int* __restrict__ fmax) {
  const int64_t base = int64_t(blockIdx.x) * 256 * kAppendPer + threadIdx.x;
  int f = -1;
  unsigned int lo = 0xFFFFFFFFu, hi = 0;
  for (int j = 0; j < kAppendPer; ++j) {
    const int64_t v = base + j * 256;
    if (v >= G.n) break;
    const int fv = G.field(int(v));
    if (fv != f) {
      if (f >= 0) {
        atomicMin(&fmin[f], lo);
        atomicMax(&fmax[f], hi);
      }
      f = fv;
      lo = 0xFFFFFFFFu;
      hi = 0;
    }
    const unsigned int r = unsigned(rank[v]);
    lo = min(lo, r);
    hi = max(hi, r);
  }
  const int f0 = __shfl(f, 0, 64);
  if (__all(f == f0) && f0 >= 0) {
    for (int sh = 32; sh >= 1; sh >>= 1) {
      lo = min(lo, unsigned(__shfl_xor(int(lo), sh, 64)));
      hi = max(hi, unsigned(__shfl_xor(int(hi), sh, 64)));
    }
    if (__lane_id() == 0) {
      atomicMin(&fmin[f0], lo);
      atomicMax(&fmax[f0], hi);
    }
  } else if (f >= 0) {
    atomicMin(&fmin[f], lo);
    atomicMax(&fmax[f], hi);
  }
}

// One essential pair per field, appended at `at`.
__global__ void k_essential(const unsigned int* __restrict__ fmin,
                            const unsigned int* __restrict__ fmax,
                            const int32_t* __restrict__ order, int nf, PairOut po, int64_t at) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t p = at + f;
  po.dim[p] = 0;
  po.birth[p] = order[fmin[f]];
  po.death[p] = -1;
  po.bkey[p] = uint64_t(fmin[f]) << 12;
  po.dkey[p] = uint64_t(fmax[f]) << 12;
}

__global__ void k_diag_keys(const int32_t* __restrict__ pdim, const uint64_t* __restrict__ bkey,
                            const uint64_t* __restrict__ dkey, int64_t np, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ idx, unsigned int* __restrict__ nd) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t rb = 0, rd = 0;
  if (i < np) {
    rb = bkey[i] >> 12;
    rd = dkey[i] >> 12;
  }
  const bool take = i < np && rb != rd;  // zero persistence is dropped
  const unsigned int p = block_append(take, nd);
  if (!take) return;
  keys[p] = (rb << 39) | (rd << 14) | (uint64_t(pdim[i]) << 12) | (bkey[i] & 0xFFFu);
  idx[p] = uint32_t(i);
}

// ======================================================================
// gradient decode (dense partner arrays)
// ======================================================================

__global__ void k_valid_cells(Grid g, int32_t* __restrict__ eup, int32_t* __restrict__ tup) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n) return;
  int x, y, z;
  coords(g, v, &x, &y, &z);
  for (int t = 0; t < 7; ++t) {
    const int m = t + 1;
    const bool ok = x + (m & 1) < g.Lx && y + ((m >> 1) & 1) < g.Ly && z + ((m >> 2) & 1) < g.Lz;
    eup[7 * v + t] = ok ? -1 : -2;
  }
  for (int t = 0; t < 12; ++t) {
    const int m = c_st.tri_chain[t][2];
    const bool ok = x + (m & 1) < g.Lx && y + ((m >> 1) & 1) < g.Ly && z + ((m >> 2) & 1) < g.Lz;
    tup[12 * v + t] = ok ? -1 : -2;
  }
}

__global__ void k_decode(Grid g, NbOff off, const int32_t* __restrict__ rank,
                         const uint4* __restrict__ code, int32_t* __restrict__ vup,
                         int32_t* __restrict__ eup, int32_t* __restrict__ tup) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n) return;
  int x, y, z;
  coords(g, v, &x, &y, &z);
  const uint32_t valid = valid_nbs(g, x, y, z);
  const int rx = rank[v];
  uint32_t low = 0;
  for (int k = 0; k < 14; ++k)
    if (((valid >> k) & 1u) && rank[v + off.o[k]] < rx) low |= 1u << k;
  const uint4 c = code[v];
  vup[v] = -1;
  auto edge_id = [&](int k) { return k < 7 ? 7 * v + k : 7 * (v + off.o[k]) + (k - 7); };
  auto tri_id = [&](int t) {
    return 12 * (v + lin(g, c_st.tri_anc[t][0], c_st.tri_anc[t][1], c_st.tri_anc[t][2])) +
           c_st.tri_type[t];
  };
  auto tet_id = [&](int q) {
    return 6 * (v + lin(g, c_st.tet_anc[q][0], c_st.tet_anc[q][1], c_st.tet_anc[q][2])) +
           c_st.tet_type[q];
  };
  for (int k = 0; k < 14; ++k) {
    if (!((low >> k) & 1u)) continue;
    const uint32_t ec = edge_code(c, k);
    if (ec == 7u) {
      vup[v] = edge_id(k);
    } else if (ec < 6u) {
      uint64_t m = c_st.edge_trim[k];
      for (uint32_t s = 0; s < ec; ++s) m &= m - 1;
      eup[edge_id(k)] = tri_id(ffs64(m));
    }
  }
  for (int t = 0; t < 36; ++t) {
    if ((uint32_t(c_st.tri_nbm[t]) & low) != uint32_t(c_st.tri_nbm[t])) continue;
    const uint32_t tc = tri_code(c, t);
    if (tc >= 2u) tup[tri_id(t)] = tet_id(c_st.tri_tet[t][tc - 2]);
  }
}

inline unsigned blocks_for(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

// An integer from the environment, clamped to [lo, hi]; dflt when unset.
inline int env_int(const char* name, int dflt, int lo, int hi) {
  const char* e = std::getenv(name);
  if (!e) return dflt;
  return std::min(hi, std::max(lo, std::atoi(e)));
}

template <class T>
T read_scalar(const T* dptr, hipStream_t s) {
  T v;
  TS_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  return v;
}

// Union-find rounds shared by K5 and K6.
int union_find_rounds(ts_ctx* ctx, int64_t nedges, int64_t nnodes, int32_t* ca, int32_t* cb,
                      uint8_t* state, int dual, const int32_t* cell_id, const uint64_t* cell_key,
                      const int32_t* node_id, const uint64_t* node_key, PairOut po,
                      const char* tag) {
  hipStream_t s = ctx->stream;
  Workspace& ws = ctx->ws;
  const std::string t(tag);
  int32_t* parent = ws.get<int32_t>(t + ".parent", nnodes + 1);
  unsigned int* best = ws.get<unsigned int>(t + ".best", nnodes + 1);
  uint32_t* listA = ws.get<uint32_t>(t + ".listA", nedges + 1);
  uint32_t* listB = ws.get<uint32_t>(t + ".listB", nedges + 1);
  unsigned int* cnt = ws.get<unsigned int>(t + ".cnt", 4);
  k_uf_init<<<blocks_for(nnodes), 256, 0, s>>>(parent, best, nnodes);
  unsigned int h_n = unsigned(nedges);
  k_fill_u32<<<1, 1, 0, s>>>(cnt, 1, h_n);
  // listA already holds 0..nedges-1 (written by the init kernel)
  int rounds = 0;
  uint32_t* cur = listA;
  uint32_t* nxt = listB;
  unsigned int* ncur = cnt;
  unsigned int* nnxt = cnt + 1;
  // The active count is read back every kUfCheck rounds only: a round's list
  // is a subset of the previous one, so grids sized by the last count read
  // cover the rounds launched before the next read, and a round over an empty
  // list changes nothing (it reads the count on the device).
  const int kUfCheck = env_int("TS_UF_CHECK", 4, 1, 64);
  while (h_n > 0) {
    const unsigned grid = blocks_for(h_n);
    for (int it = 0; it < kUfCheck; ++it) {
      ++rounds;
      k_fill_u32<<<1, 1, 0, s>>>(nnxt, 1, 0u);
      k_uf_hook<<<grid, 256, 0, s>>>(cur, ncur, ca, cb, parent, best, state, dual, nedges);
      k_uf_link<<<grid, 256, 0, s>>>(cur, ncur, ca, cb, parent, best, state, nxt, nnxt, dual,
                                     nedges, cell_id, cell_key, node_id, node_key, po);
      k_uf_reset<<<blocks_for(nnodes), 256, 0, s>>>(parent, best, nnodes);
      std::swap(cur, nxt);
      std::swap(ncur, nnxt);
    }
    TS_HIP(hipGetLastError());
    h_n = read_scalar(ncur, s);
    if (rounds > nedges + 2 + kUfCheck) throw Error(TS_ERR_INTERNAL, "union-find did not converge");
  }
  return rounds;
}

}  // namespace

// ======================================================================
// Host orchestration
// ======================================================================

void compute_order(ts_ctx* ctx, const float* f, int n, int32_t* order, int32_t* rank) {
  hipStream_t s = ctx->stream;
  Workspace& ws = ctx->ws;
  uint32_t* keys = ws.get<uint32_t>("ord.keys", n);
  uint32_t* vals = ws.get<uint32_t>("ord.vals", n);
  int* bad = ws.get<int>("ord.bad", 1);
  TS_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  ctx->timer.start("K1 order keys");
  k_order_keys<<<blocks_for(n), 256, 0, s>>>(f, n, keys, vals, bad);
  ctx->timer.stop();
  ctx->timer.start("K1 radix sort");
  radix_sort_u32(ws, keys, vals, n, 0, 32, s);
  ctx->timer.stop();
  ctx->timer.start("K2 rank");
  k_rank_scatter<<<blocks_for(n), 256, 0, s>>>(vals, n, rank, order);
  ctx->timer.stop();
  TS_HIP(hipGetLastError());
  if (read_scalar(bad, s)) throw Error(TS_ERR_NONFINITE, "field contains NaN or Inf");
}

// ---------------------------------------------------------------- vertex
// order without allocation.  Its temporaries (sort keys and values, their
// ping-pong buffers, digit histograms, scan sums, the non-finite flag) live
// in one static device array, sized for kNoAllocMaxN vertices: 16 bytes per
// vertex plus 1 MiB.  Every device that runs it holds its own copy of the
// array until the process ends; its address is taken once per device with
// hipGetSymbolAddress (the array's name is not a device address in host
// code).  Calls that overlap on one device share the array and race.
constexpr int64_t kNoAllocMaxN = int64_t(1) << 21;
constexpr size_t kNoAllocScratchBytes = size_t(kNoAllocMaxN) * 16 + (size_t(1) << 20);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

__global__ void k_clear_flag(int* flag) { *flag = 0; }

// The array's device address on the current device (taken on the first call there).
char* scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  TS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(TS_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    TS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(TS_ERR_HIP, "no device address for the scratch array");
    addr[dev] = p;
  }
  return static_cast<char*>(addr[dev]);
}

void order_noalloc(const float* f, int64_t n, int32_t* order, int32_t* rank, hipStream_t s) {
  if (!f || !order || !rank || n < 1) throw Error(TS_ERR_ARG, "bad arguments");
  if (n > kNoAllocMaxN)
    throw Error(TS_ERR_ARG, "more than 2^21 vertices: beyond the no-allocation scratch");
  Arena a;
  a.base = scratch_address();
  a.cap = kNoAllocScratchBytes;
  uint32_t* keys = a.get<uint32_t>("keys", size_t(n));
  uint32_t* vals = a.get<uint32_t>("vals", size_t(n));
  int* bad = a.get<int>("bad", 1);
  k_clear_flag<<<1, 1, 0, s>>>(bad);
  k_order_keys<<<blocks_for(int(n)), 256, 0, s>>>(f, int(n), keys, vals, bad);
  TS_HIP(hipGetLastError());
  radix_sort_u32(a, keys, vals, size_t(n), 0, 32, s);
  k_rank_scatter<<<blocks_for(int(n)), 256, 0, s>>>(vals, int(n), rank, order);
  TS_HIP(hipGetLastError());
  if (read_scalar(bad, s)) throw Error(TS_ERR_NONFINITE, "field contains NaN or Inf");
}

void compute_persistence(ts_ctx* ctx, const float* f, const Grid& g, PersistenceResult* R,
                         const uint8_t* changed, const Batch* batch) {
  upload_tables(ctx->device);
  hipStream_t s = ctx->stream;
  const bool trace = std::getenv("TS_TRACE") != nullptr;
  if (trace) TS_HIP(hipStreamSynchronize(s));
  const auto t_wall = std::chrono::steady_clock::now();
  Workspace& ws = ctx->ws;
  const int n = g.n;
  const int nf = batch ? int(batch->grids.size()) : 1;
  std::vector<int64_t> layout;
  if (batch) {
    if (nf < 1 || int64_t(batch->base.size()) != nf + 1 || batch->base[nf] != n)
      throw Error(TS_ERR_ARG, "batch layout does not match the vertex count");
    for (int i = 0; i < nf; ++i) {
      const Grid& h = batch->grids[i];
      if (batch->base[i + 1] - batch->base[i] != int64_t(h.n) || h.n < 1)
        throw Error(TS_ERR_ARG, "batch field sizes do not match their grids");
      layout.insert(layout.end(), {h.Lx, h.Ly, h.Lz});
    }
  } else {
    layout = {g.Lx, g.Ly, g.Lz};
  }
  const bool update = changed != nullptr && R->complete && R->g.n == g.n && R->layout == layout;
  R->complete = false;
  R->g = g;
  R->layout = layout;
  R->nfields = nf;
  R->order = ws.get<int32_t>("pm.order", n);
  R->rank = ws.get<int32_t>("pm.rank", n);
  R->code = ws.get<uint4>("pm.code", n);
  R->down = ws.get<int32_t>("pm.down", n);
  // the previous order and critical lists, read by the fast update
  int32_t* prev_order = nullptr;
  uint64_t* prev_key[4] = {};
  int32_t* prev_id[4] = {};
  int64_t prev_n[4] = {0, 0, 0, 0};
  if (update) {
    prev_order = ws.get<int32_t>("pm.order_prev", n);
    TS_HIP(hipMemcpyAsync(prev_order, R->order, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    for (int d = 0; d < 4; ++d) {
      prev_n[d] = R->ncrit[d];
      prev_key[d] = ws.get<uint64_t>("pm.ckey_prev" + std::to_string(d), prev_n[d] + 1);
      prev_id[d] = ws.get<int32_t>("pm.cid_prev" + std::to_string(d), prev_n[d] + 1);
      if (prev_n[d] > 0) {
        TS_HIP(hipMemcpyAsync(prev_key[d], R->ckey[d], size_t(prev_n[d]) * 8,
                              hipMemcpyDeviceToDevice, s));
        TS_HIP(hipMemcpyAsync(prev_id[d], R->cid[d], size_t(prev_n[d]) * 4,
                              hipMemcpyDeviceToDevice, s));
      }
    }
  }
  compute_order(ctx, f, n, R->order, R->rank);

  // geometry: one grid, or a batch resolved through a field table and a page map
  GeoOne G1{g, batch ? NbOff{} : make_offsets(g)};
  GeoBatch GB{nullptr, nullptr, nf, n};
  if (batch) {
    std::vector<FieldDesc> hfd(nf);
    for (int i = 0; i < nf; ++i) {
      const Grid& h = batch->grids[i];
      const NbOff o = make_offsets(h);
      hfd[i].base = int(batch->base[i]);
      hfd[i].Lx = h.Lx;
      hfd[i].Ly = h.Ly;
      hfd[i].Lz = h.Lz;
      for (int k = 0; k < 14; ++k) hfd[i].o[k] = o.o[k];
    }
    const int64_t npages = (int64_t(n) + (1 << kPageBits) - 1) >> kPageBits;
    std::vector<int32_t> hpage(npages);
    for (int i = 0, p = 0; p < npages; ++p) {
      const int64_t first = int64_t(p) << kPageBits;
      while (i + 1 < nf && first >= batch->base[i + 1]) ++i;
      hpage[p] = i;
    }
    FieldDesc* dfd = ws.get<FieldDesc>("pm.fields", nf);
    int32_t* dpage = ws.get<int32_t>("pm.pages", npages);
    TS_HIP(hipMemcpyAsync(dfd, hfd.data(), nf * sizeof(FieldDesc), hipMemcpyHostToDevice, s));
    TS_HIP(hipMemcpyAsync(dpage, hpage.data(), npages * 4, hipMemcpyHostToDevice, s));
    TS_HIP(hipStreamSynchronize(s));
    GB.fd = dfd;
    GB.page = dpage;
  }
  auto with_geo = [&](auto&& fn) {
    if (batch) fn(GB);
    else fn(G1);
  };

  // dirty vertices of the fast update
  uint8_t* dirty = nullptr;
  uint32_t* dlist = nullptr;
  int64_t ndirty = n;
  if (update) {
    dirty = ws.get<uint8_t>("pm.dirty", n);
    dlist = ws.get<uint32_t>("pm.dirty_list", n);
    unsigned long long* dcnt = ws.get<unsigned long long>("pm.dirty_count", 1);
    TS_HIP(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long), s));
    ctx->timer.start("K3 dirty");
    with_geo([&](auto G) {
      k_dirty<<<blocks_for(n, 256 * kAppendPer), 256, 0, s>>>(changed, G, dirty, dlist, dcnt);
    });
    ctx->timer.stop();
    TS_HIP(hipGetLastError());
    unsigned long long h = 0;
    TS_HIP(hipMemcpyAsync(&h, dcnt, sizeof(h), hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    ndirty = int64_t(h);
    if (ndirty > n) throw Error(TS_ERR_INTERNAL, "dirty vertex count exceeds the grid");
  }
  R->n_regrad = ndirty;

  // ---- K3 + K4: gradient and critical cells ----
  unsigned long long* ccount = ws.get<unsigned long long>("pm.ccount", 4);
  static int64_t cap_hint[4] = {0, 0, 0, 0};
  int64_t cap[4];
  for (int d = 0; d < 4; ++d) cap[d] = std::max<int64_t>(cap_hint[d], std::max<int64_t>(1024, n / 4));
  // TS_CRIT_CAP: start from a given list capacity (exercises the retry path)
  if (const char* e = std::getenv("TS_CRIT_CAP"))
    for (int d = 0; d < 4; ++d) cap[d] = std::max<int64_t>(1, std::atoll(e));
  for (int attempt = 0; attempt < 3; ++attempt) {
    CritOut co;
    for (int d = 0; d < 4; ++d) {
      co.key[d] = ws.get<uint64_t>("pm.ckey" + std::to_string(d), cap[d]);
      co.id[d] = ws.get<int32_t>("pm.cid" + std::to_string(d), cap[d]);
      co.cap[d] = cap[d];
    }
    co.count = ccount;
    TS_HIP(hipMemsetAsync(ccount, 0, 4 * sizeof(unsigned long long), s));
    if (update) {
      ctx->timer.start("K3 keep");
      for (int d = 0; d < 4; ++d)
        if (prev_n[d] > 0)
          k_keep_crit<<<blocks_for(prev_n[d], 256 * kAppendPer), 256, 0, s>>>(
              prev_key[d], prev_id[d], prev_n[d], prev_order, R->rank, dirty, co.key[d],
              co.id[d], co.cap[d], ccount + d);
      ctx->timer.stop();
      TS_HIP(hipGetLastError());
      if (ndirty > 0) {
        ctx->timer.start("K3 gradient (dirty)");
        with_geo([&](auto G) {
          k_gradient<true><<<blocks_for(ndirty, kGradThreads), kGradThreads, 0, s>>>(
              R->rank, G, R->code, R->down, co, dlist, ndirty);
        });
        ctx->timer.stop();
      }
    } else {
      // persistent workgroups over a queue of 3D tiles (or of runs of
      // consecutive vertex ids, the last candidate); the shape is picked by
      // the launch tuner per size class (every shape gives the same
      // gradient), or fixed by TS_K3_TILE (index into the candidates)
      static const int kTiles[7][3] = {{256, 1, 1}, {64, 4, 1}, {32, 8, 1}, {32, 4, 2},
                                       {16, 4, 4},  {8, 8, 4},  {0, 0, 0}};
      const std::string tkey = std::string(batch ? "k3.tiles.batch." : "k3.tiles.") +
                               std::to_string(64 - __builtin_clzll(uint64_t(n) | 1));
      int tidx = -1, shape = 0;
      if (std::getenv("TS_K3_TILE")) {
        shape = env_int("TS_K3_TILE", 0, 0, 6);
      } else {
        tidx = ctx->tuner.pick(tkey, 7);
        shape = tidx;
      }
      const int tx = kTiles[shape][0], ty = kTiles[shape][1], tz = kTiles[shape][2];
      std::vector<int4> hf;
      std::vector<int64_t> htb(1, 0);
      auto add_field = [&](int base, int Lx, int Ly, int Lz) {
        hf.push_back(make_int4(base, Lx, Ly, Lz));
        htb.push_back(htb.back() + int64_t((Lx + tx - 1) / tx) * ((Ly + ty - 1) / ty) *
                                      ((Lz + tz - 1) / tz));
      };
      if (tx == 0) {
        hf.push_back(make_int4(0, 0, 0, 0));
        htb.push_back((n + kGradThreads - 1) / kGradThreads);
      } else if (batch) {
        for (int i = 0; i < nf; ++i)
          add_field(int(batch->base[i]), batch->grids[i].Lx, batch->grids[i].Ly,
                    batch->grids[i].Lz);
      } else {
        add_field(0, g.Lx, g.Ly, g.Lz);
      }
      int4* dfield = ws.get<int4>("pm.k3.fields", hf.size());
      int64_t* dtb = ws.get<int64_t>("pm.k3.tile_base", htb.size());
      unsigned int* dhead = ws.get<unsigned int>("pm.k3.head", kTileQueues);
      TS_HIP(hipMemcpyAsync(dfield, hf.data(), hf.size() * sizeof(int4), hipMemcpyHostToDevice, s));
      TS_HIP(hipMemcpyAsync(dtb, htb.data(), htb.size() * 8, hipMemcpyHostToDevice, s));
      k_fill_u32<<<1, kTileQueues, 0, s>>>(dhead, kTileQueues, 0u);
      TileQueue q{dfield, dtb, int(hf.size()), tx, ty, tz, dhead, htb.back()};
      static int n_cu = 0;
      if (!n_cu) {
        TS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
        n_cu = std::max(n_cu, 1);
      }
      // workgroups resident at once (the kernel's LDS allows 4 per CU)
      const unsigned grid = unsigned(std::min<int64_t>(q.nitems, int64_t(4) * n_cu));
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (tidx >= 0) {
        TS_HIP(hipEventCreate(&e0));
        TS_HIP(hipEventCreate(&e1));
        TS_HIP(hipEventRecord(e0, s));
      }
      ctx->timer.start("K3 gradient");
      if (grid > 0)
        with_geo([&](auto G) {
          k_gradient_tiles<<<grid, kGradThreads, 0, s>>>(R->rank, G, R->code, R->down, co, q);
        });
      ctx->timer.stop();
      TS_HIP(hipGetLastError());
      if (tidx >= 0) {
        TS_HIP(hipEventRecord(e1, s));
        TS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TS_HIP(hipEventElapsedTime(&ms, e0, e1));
        ctx->tuner.report(tkey, tidx, double(ms) * 1e-3);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
      }
    }
    TS_HIP(hipGetLastError());
    unsigned long long h[4];
    TS_HIP(hipMemcpyAsync(h, ccount, sizeof(h), hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    bool fits = true;
    for (int d = 0; d < 4; ++d) {
      R->ncrit[d] = int64_t(h[d]);
      if (R->ncrit[d] > cap[d]) {
        fits = false;
        cap[d] = R->ncrit[d] + R->ncrit[d] / 8 + 1024;
      }
      cap_hint[d] = std::max(cap_hint[d], cap[d]);
    }
    if (fits) {
      for (int d = 0; d < 4; ++d) {
        R->ckey[d] = co.key[d];
        R->cid[d] = co.id[d];
      }
      break;
    }
    if (attempt == 2) throw Error(TS_ERR_INTERNAL, "critical-cell buffers did not fit");
  }
  if (R->ncrit[0] - R->ncrit[1] + R->ncrit[2] - R->ncrit[3] != nf)
    throw Error(TS_ERR_INTERNAL, "Euler characteristic of the critical cells is not 1");
  const int64_t nmin = R->ncrit[0], ne = R->ncrit[1], ntri = R->ncrit[2], nmax = R->ncrit[3];

  // sort every list by key; keep an id-sorted index for lookups
  ctx->timer.start("K4 sort critical");
  const int keybits = 12 + 32 - __builtin_clz(uint32_t(std::max(n - 1, 1)));
  for (int d = 0; d < 4; ++d) {
    if (R->ncrit[d] <= 1) continue;
    uint32_t* perm = ws.get<uint32_t>("pm.perm", R->ncrit[d]);
    k_iota<<<blocks_for(R->ncrit[d]), 256, 0, s>>>(perm, R->ncrit[d]);
    radix_sort_u64(ws, R->ckey[d], perm, R->ncrit[d], 0, keybits, s);
    int32_t* ids2 = ws.get<int32_t>("pm.cid_sorted" + std::to_string(d), R->ncrit[d]);
    k_gather_ids<<<blocks_for(R->ncrit[d]), 256, 0, s>>>(R->cid[d], perm, R->ncrit[d],
                                                         reinterpret_cast<uint32_t*>(ids2));
    R->cid[d] = ids2;
  }
  // id -> position maps for edges (rows) and tets (maxima)
  int32_t* edge_pos_of = ws.get<int32_t>("pm.edge_pos_of", int64_t(7) * n);
  int32_t* max_pos_of = ws.get<int32_t>("pm.max_pos_of", int64_t(6) * n);
  if (R->ncrit[1] > 0)
    k_pos_map<<<blocks_for(R->ncrit[1]), 256, 0, s>>>(R->cid[1], R->ncrit[1], edge_pos_of);
  if (R->ncrit[3] > 0)
    k_pos_map<<<blocks_for(R->ncrit[3]), 256, 0, s>>>(R->cid[3], R->ncrit[3], max_pos_of);
  ctx->timer.stop();

  // pair output
  const int64_t pcap = nmin + nmax + ne + nf + 16;
  PairOut po;
  po.dim = ws.get<int32_t>("pm.pdim", pcap);
  po.birth = ws.get<int32_t>("pm.pbirth", pcap);
  po.death = ws.get<int32_t>("pm.pdeath", pcap);
  po.bkey = ws.get<uint64_t>("pm.pbkey", pcap);
  po.dkey = ws.get<uint64_t>("pm.pdkey", pcap);
  po.count = ws.get<unsigned long long>("pm.pcount", 1);
  po.cap = pcap;
  TS_HIP(hipMemsetAsync(po.count, 0, sizeof(unsigned long long), s));
  int* err = ws.get<int>("pm.err", 1);
  TS_HIP(hipMemsetAsync(err, 0, sizeof(int), s));

  // ---- K5: min-saddle ----
  uint8_t* estate = ws.get<uint8_t>("pm.estate", ne + 1);
  if (ne > 0) {
    ctx->timer.start("K5 d0 paths");
    int32_t* min_idx = ws.get<int32_t>("pm.minidx", n);
    int32_t* ca = ws.get<int32_t>("pm.ca", ne);
    int32_t* cb = ws.get<int32_t>("pm.cb", ne);
    uint32_t* listA = ws.get<uint32_t>("uf0.listA", ne + 1);
    k_min_index<<<blocks_for(nmin), 256, 0, s>>>(R->cid[0], nmin, min_idx);
    k_fill_u8<<<blocks_for(ne), 256, 0, s>>>(estate, ne, 0);
    with_geo([&](auto G) {
      k_d0_init<<<blocks_for(ne), 256, 0, s>>>(R->cid[1], ne, G, R->down, min_idx, ca, cb, listA,
                                               err);
    });
    ctx->timer.stop();
    ctx->timer.start("K5 d0 union-find");
    R->rounds_d0 = union_find_rounds(ctx, ne, nmin, ca, cb, estate, 0, R->cid[1], R->ckey[1],
                                     R->cid[0], R->ckey[0], po, "uf0");
    ctx->timer.stop();
  }

  // ---- K6: saddle-max ----
  uint8_t* tstate = ws.get<uint8_t>("pm.tstate", ntri + 1);
  if (ntri > 0) {
    ctx->timer.start("K6 d2 paths");
    int32_t* ca = ws.get<int32_t>("pm.ca", std::max(ne, ntri));
    int32_t* cb = ws.get<int32_t>("pm.cb", std::max(ne, ntri));
    uint32_t* listA = ws.get<uint32_t>("uf2.listA", ntri + 1);
    k_fill_u8<<<blocks_for(ntri), 256, 0, s>>>(tstate, ntri, 0);
    with_geo([&](auto G) {
      k_d2_init<<<blocks_for(ntri), 256, 0, s>>>(R->cid[2], R->ckey[2], ntri, G, R->order,
                                                 R->code, max_pos_of, R->cid[3], nmax,
                                                 ca, cb, listA, err);
    });
    ctx->timer.stop();
    ctx->timer.start("K6 d2 union-find");
    // node ids/keys of maxima; the outside (index nmax) never dies
    R->rounds_d2 = union_find_rounds(ctx, ntri, nmax + 1, ca, cb, tstate, 1, R->cid[2],
                                     R->ckey[2], R->cid[3], R->ckey[3], po, "uf2");
    ctx->timer.stop();
  }
  {
    const int h_err = read_scalar(err, s);
    if (h_err) throw Error(TS_ERR_INTERNAL, "gradient path error " + std::to_string(h_err));
  }

  // ---- K7: saddle-saddle ----
  if (ne > 0)
    k_pos_drop<<<blocks_for(ne), 256, 0, s>>>(R->cid[1], estate, ne, edge_pos_of);
  unsigned int* ncols_d = ws.get<unsigned int>("d1.ncols", 1);
  TS_HIP(hipMemsetAsync(ncols_d, 0, sizeof(unsigned int), s));
  uint32_t* cols = ws.get<uint32_t>("d1.cols", ntri + 1);
  if (ntri > 0) {
    k_collect_cols<<<blocks_for(ntri), 256, 0, s>>>(tstate, ntri, cols, ncols_d);
  }
  const int64_t ncols = read_scalar(ncols_d, s);
  if (ncols > 0) {
    // columns in increasing key order
    ctx->timer.start("K7 d1 boundary");
    {
      uint32_t* ckeys = ws.get<uint32_t>("d1.ckeys", ncols);
      TS_HIP(hipMemcpyAsync(ckeys, cols, ncols * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      radix_sort_u32(ws, ckeys, cols, ncols, 0, 32, s);
    }
    uint64_t* col_desc = ws.get<uint64_t>("d1.desc", ncols);
    k_fill_u64<<<blocks_for(ncols), 256, 0, s>>>(col_desc, ncols, ~0ull);
    static int64_t pool_hint = 0;
    int64_t pool_cap = std::max<int64_t>(pool_hint, std::max<int64_t>(1 << 20, 16 * ncols));
    // TS_D1_POOL_WORDS: start from a given pool size (exercises the growth paths)
    if (const char* e = std::getenv("TS_D1_POOL_WORDS")) pool_cap = std::max<int64_t>(64, std::atoll(e));
    ColPool pool;
    pool.data = ws.get<uint32_t>("d1.pool", pool_cap);
    pool.top = ws.get<unsigned long long>("d1.top", 1);
    pool.cap = pool_cap;
    TS_HIP(hipMemsetAsync(pool.top, 0, sizeof(unsigned long long), s));
    uint32_t* todo[2] = {ws.get<uint32_t>("d1.todoA", ncols + 1),
                         ws.get<uint32_t>("d1.todoB", ncols + 1)};
    unsigned int* nretry = ws.get<unsigned int>("d1.nretry", 1);
    int* bfull = ws.get<int>("d1.bfull", 1);
    BoundaryCommon BA;
    BA.cols = cols;
    BA.tri_ids = R->cid[2];
    BA.tri_keys = R->ckey[2];
    BA.rank = R->rank;
    BA.order = R->order;
    BA.code = R->code;
    BA.edge_pos_of = edge_pos_of;
    BA.edge_ids = R->cid[1];
    BA.nedges = ne;
    BA.nretry = nretry;
    BA.pool_full = bfull;
    BA.err = err;
    BA.stats = nullptr;
    // launch parameters, overridable for tuning (TS_D1_*); results do not depend on them
    const int pass0_steps = env_int("TS_D1_STEPS", 512, 16, 1 << 20);
    BA.wave_cap = env_int("TS_D1_WAVE_CAP", WaveListR<kWaveRegs>::kCap, 4, WaveListR<kWaveRegs>::kCap);
    BA.wave2_cap =
        env_int("TS_D1_WAVE2_CAP", WaveListR<kWaveRegs2>::kCap, 4, WaveListR<kWaveRegs2>::kCap);
    int64_t ntodo = ncols;
    const uint32_t* list = nullptr;  // first pass: every column
    for (int pass = 0, kind = 0;; ++pass) {
      // kind 0 (every column): one lane per column, a small heap in LDS and
      // a bounded number of pops; kind 1: the rest, one column per wave, the
      // queue in the wave's registers (256 entries); kind 2: columns whose
      // queue outgrows that, the same with 1024 entries; kind 3: columns
      // whose queue outgrows that too, one column per wave with a large heap
      // in LDS
      const bool lds = kind >= 1;
      uint32_t* out = todo[pass & 1];
      TS_HIP(hipMemsetAsync(nretry, 0, sizeof(unsigned int), s));
      TS_HIP(hipMemsetAsync(bfull, 0, sizeof(int), s));
      if (std::getenv("TS_TRACE")) {
        BA.stats = ws.get<unsigned long long>("d1.bstats", 40);
        k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<uint64_t*>(BA.stats), 40, 0);
      }
      BA.pool = pool;
      BA.col_desc = col_desc;
      BA.retry = out;
      BA.max_steps = lds ? 64 * g.n : pass0_steps;
      if (kind == 0) {
        const unsigned nb = unsigned(std::min<int64_t>((ntodo + kLaneThreads - 1) / kLaneThreads, 8192));
        with_geo([&](auto G) {
          BoundaryArgs<decltype(G)> A;
          static_cast<BoundaryCommon&>(A) = BA;
          A.G = G;
          k_d1_boundary_lanes<<<nb, kLaneThreads, 0, s>>>(A, list, ntodo);
        });
      } else {
        const unsigned nb = unsigned(std::min<int64_t>(ntodo, 8192));
        with_geo([&](auto G) {
          BoundaryArgs<decltype(G)> A;
          static_cast<BoundaryCommon&>(A) = BA;
          A.G = G;
          if (kind == 1 || kind == 2) {
            unsigned int* next = ws.get<unsigned int>("d1.bnext", 1);
            k_fill_u32<<<1, 1, 0, s>>>(next, 1, 0u);
            if (kind == 1)
              k_d1_boundary_wave<decltype(G), kWaveRegs><<<nb, 64, 0, s>>>(A, list, ntodo, next);
            else
              k_d1_boundary_wave<decltype(G), kWaveRegs2><<<nb, 64, 0, s>>>(A, list, ntodo, next);
          } else {
            k_d1_boundary_lds<<<nb, 64, 0, s>>>(A, list, ntodo);
          }
        });
      }
      TS_HIP(hipGetLastError());
      if (BA.stats) {
        unsigned long long h[40];
        TS_HIP(hipMemcpyAsync(h, BA.stats, sizeof(h), hipMemcpyDeviceToHost, s));
        TS_HIP(hipStreamSynchronize(s));
        std::fprintf(stderr,
                     "[topsimp] d1 boundary pass %d: columns %lld %s steps %llu max %llu max heap "
                     "%llu long %llu retried %llu; log2 histogram:",
                     pass, (long long)ntodo,
                     kind == 0 ? "lanes" : (kind == 1 ? "wave" : (kind == 2 ? "wave1024" : "lds")),
                     h[0], h[1], h[2], h[3], h[4]);
        for (int b = 0; b < 21; ++b) std::fprintf(stderr, " %llu", h[5 + b]);
        std::fprintf(stderr, "; largest heap <= 8, 16, 32, 64, 128, more:");
        for (int b = 0; b < 6; ++b) std::fprintf(stderr, " %llu", h[26 + b]);
        std::fprintf(stderr,
                     "; toggles %llu rows moved %llu vertex groups %llu expansions %llu; columns "
                     "over 2000 pops: pops %llu toggles %llu moved %llu groups %llu\n",
                     h[32], h[33], h[34], h[35], h[36], h[37], h[38], h[39]);
      }
      ntodo = read_scalar(nretry, s);
      if (ntodo == 0) break;
      if (pass > 12) throw Error(TS_ERR_INTERNAL, "boundary extraction did not finish");
      list = out;
      const int done_kind = kind;
      kind = std::min(kind + 1, 3);
      if (kind <= 2 && ntodo > 1) {
        // the wave passes take their columns in order from a shared counter:
        // the highest columns, whose expansions are the longest, go first so
        // that they do not start after the bulk and set the pass's length
        uint32_t* keys = ws.get<uint32_t>("d1.retry_keys", ncols + 1);
        k_desc_keys<<<blocks_for(ntodo), 256, 0, s>>>(list, ntodo, uint32_t(ncols - 1), keys);
        int bits = 1;
        while (bits < 32 && (uint64_t(1) << bits) < uint64_t(ncols)) ++bits;
        radix_sort_u32(ws, keys, out, size_t(ntodo), 0, bits, s);
      }
      if (read_scalar(bfull, s)) {
        // grow the pool keeping its contents
        // (failed reservations past the old capacity were never written)
        const int64_t keep = std::min<int64_t>(int64_t(read_scalar(pool.top, s)), pool_cap);
        const int64_t ncap = std::max<int64_t>(2 * pool_cap, keep + 8 * ntodo);
        uint32_t* np = ws.get<uint32_t>("d1.pool2", ncap);
        TS_HIP(hipMemcpyAsync(np, pool.data, keep * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        std::swap(ws.bufs["d1.pool"], ws.bufs["d1.pool2"]);
        pool.data = np;
        pool_cap = ncap;
        pool.cap = ncap;
        k_set_u64<<<1, 1, 0, s>>>(pool.top, uint64_t(keep));
        TS_HIP(hipGetLastError());
      } else if (done_kind == 3) {
        throw Error(TS_ERR_CAPACITY, "saddle-saddle boundary exceeds the LDS heap");
      }
    }
    pool_hint = std::max(pool_hint, pool_cap);
    ctx->timer.stop();
    auto length_stats = [&](const char* what) {
      if (!std::getenv("TS_TRACE")) return;
      std::vector<uint64_t> desc(ncols);
      TS_HIP(hipMemcpy(desc.data(), col_desc, ncols * 8, hipMemcpyDeviceToHost));
      std::vector<uint32_t> L(ncols);
      uint64_t tot = 0;
      for (int64_t c = 0; c < ncols; ++c) tot += (L[c] = uint32_t(desc[c] & 0xFFFFFFu));
      std::sort(L.begin(), L.end());
      std::fprintf(stderr,
                   "[topsimp] %s column lengths: mean %.2f median %u p99 %u p99.99 %u max %u\n",
                   what, double(tot) / ncols, L[ncols / 2], L[ncols * 99 / 100],
                   L[std::min<int64_t>(ncols - 1, ncols * 9999 / 10000)], L[ncols - 1]);
    };
    length_stats("boundary");

    ctx->timer.start("K7 d1 reduction");
    unsigned int* owner = ws.get<unsigned int>("d1.owner", ne + 1);
    uint64_t* pdesc = ws.get<uint64_t>("d1.pdesc", ne + 1);
    uint4* prow = ws.get<uint4>("d1.prow", 2 * (ne + 1));
    unsigned int* mark = ws.get<unsigned int>("d1.mark", ncols + 1);
    uint32_t* listA = ws.get<uint32_t>("d1.listA", ncols + 1);
    uint32_t* listB = ws.get<uint32_t>("d1.listB", ncols + 1);
    unsigned int* cnt = ws.get<unsigned int>("d1.cnt", 6);
    uint32_t* wave_list = ws.get<uint32_t>("d1.wave", ncols + 1);
    uint32_t* long_list = ws.get<uint32_t>("d1.long", ncols + 1);
    int* pool_full = ws.get<int>("d1.full", 1);
    k_fill_u32<<<blocks_for(ne), 256, 0, s>>>(owner, ne, 0xFFFFFFFFu);
    // grows the pool, compacting the live columns on the device
    int grows = 0;
    auto grow_pool = [&]() {
      ++grows;
      uint32_t* lens = ws.get<uint32_t>("d1.lens", ncols + 1);
      uint32_t* offs = ws.get<uint32_t>("d1.offs", ncols + 1);
      k_col_lengths<<<blocks_for(ncols + 1), 256, 0, s>>>(col_desc, ncols, lens);
      scan_exclusive_u32(ws, lens, offs, ncols + 1, s);  // lens[ncols] = 0: offs[ncols] = total
      const int64_t live = int64_t(read_scalar(offs + ncols, s));
      const int64_t ncap = std::max<int64_t>(2 * pool_cap, 4 * live + (1 << 20));
      if (ncap >= (int64_t(1) << 40)) throw Error(TS_ERR_INTERNAL, "column pool too large");
      uint32_t* np = ws.get<uint32_t>("d1.pool2", ncap);
      k_col_compact<<<blocks_for(ncols), 256, 0, s>>>(col_desc, ncols, pool.data, offs, np);
      std::swap(ws.bufs["d1.pool"], ws.bufs["d1.pool2"]);
      pool.data = np;
      pool_cap = ncap;
      pool.cap = ncap;
      k_set_u64<<<1, 1, 0, s>>>(pool.top, uint64_t(live));
      // owners' columns moved: publish them again
      k_d1_publish<<<blocks_for(ncols), 256, 0, s>>>(col_desc, pool.data, owner, nullptr, nullptr,
                                                     ncols, pdesc, prow);
      TS_HIP(hipGetLastError());
      pool_hint = std::max(pool_hint, pool_cap);
    };
    const int kCheckEvery = env_int("TS_D1_CHECK", 8, 1, 256);
    // Columns are reduced block by block in index order; a block's columns
    // only interact with each other once every earlier column is final.
    // the block size is autotuned per size class of the column count (the
    // pairs do not depend on it); TS_D1_BLOCK_BITS fixes it
    // (24 bits: every column in one block, so the last columns start their
    // chains as soon as their owners are final)
    static const int kBlockBits[5] = {16, 17, 18, 20, 24};
    const std::string tune_key = "d1.block." + std::to_string(64 - __builtin_clzll(uint64_t(ncols) | 1));
    int tune_idx = -1, block_bits = 16;
    if (std::getenv("TS_D1_BLOCK_BITS")) {
      block_bits = env_int("TS_D1_BLOCK_BITS", 16, 10, 24);
    } else {
      tune_idx = ctx->tuner.pick(tune_key, 5);
      block_bits = kBlockBits[tune_idx];
    }
    const int64_t kBlock = int64_t(1) << block_bits;
    const auto t_reduce = std::chrono::steady_clock::now();
    unsigned int* round_d = ws.get<unsigned int>("d1.round", 1);
    k_fill_u32<<<1, 1, 0, s>>>(round_d, 1, 1u);  // active members carry the round in mark[]
    int rounds = 0;
    uint32_t* A = listA;
    uint32_t* B = listB;
    unsigned long long* rstats = nullptr;
    if (std::getenv("TS_TRACE")) {
      rstats = ws.get<unsigned long long>("d1.rstats", 16);
      k_fill_u64<<<1, 16, 0, s>>>(reinterpret_cast<uint64_t*>(rstats), 16, 0);
    }
    for (int64_t lo = 0; lo < ncols; lo += kBlock) {
      const int64_t hi = std::min<int64_t>(ncols, lo + kBlock);
      unsigned int h_n = unsigned(hi - lo);
      k_iota_from<<<blocks_for(h_n), 256, 0, s>>>(A, h_n, uint32_t(lo));
      k_fill_u32<<<1, 1, 0, s>>>(cnt, 1, h_n);
      k_set_marks<<<blocks_for(h_n), 256, 0, s>>>(mark + lo, h_n, round_d);
      k_d1_round_begin<<<1, 1, 0, s>>>(cnt);
      while (h_n > 0) {
        // grids sized by the last known active count (the kernels stride over
        // the device-side count, so a later, larger list is still covered)
        const unsigned grid = std::min<unsigned>(std::max<unsigned>(blocks_for(h_n), 8u), 1024u);
        const unsigned lgrid =
            std::min<unsigned>(std::max<unsigned>((h_n + kRedLanes - 1) / kRedLanes, 8u), 8192u);
        const unsigned wgrid = 512u;  // the deferred columns are few (counted on the device)
        TS_HIP(hipMemsetAsync(pool_full, 0, sizeof(int), s));
        for (int it = 0; it < kCheckEvery; ++it) {
          ++rounds;
          k_d1_claim<<<grid, 256, 0, s>>>(col_desc, pool.data, owner, mark, round_d, A, cnt);
          k_d1_publish<<<grid, 256, 0, s>>>(col_desc, pool.data, owner, A, cnt, 0, pdesc, prow);
          k_d1_reduce_lanes<<<lgrid, kRedLanes, 0, s>>>(col_desc, pool.data, pool, owner, pdesc, prow, mark,
                                                          round_d, A, B, cnt, err, pool_full,
                                                          wave_list, rstats);
          k_d1_reduce_wave<<<wgrid, 64 * kRedWaves, 0, s>>>(col_desc, pool.data, pool, owner, pdesc,
                                                            prow, mark,
                                                            round_d, wave_list, B, cnt, err, pool_full,
                                                            long_list, rstats);
          k_d1_reduce_long<<<64, kLongThreads, 0, s>>>(col_desc, pool.data, pool, owner, pdesc,
                                                       prow, mark,
                                                       round_d, long_list, B, cnt, err, pool_full,
                                                       rstats);
          k_d1_round_next<<<1, 1, 0, s>>>(cnt, round_d);
          std::swap(A, B);
        }
        TS_HIP(hipGetLastError());
        h_n = read_scalar(cnt, s);
        if (std::getenv("TS_TRACE_D1")) {
          static auto t_prev = std::chrono::steady_clock::now();
          const auto t_now = std::chrono::steady_clock::now();
          std::fprintf(stderr, "[d1] block %lld rounds %d active %u  %.3f ms\n", (long long)(lo / kBlock),
                       rounds, h_n,
                       std::chrono::duration<double, std::milli>(t_now - t_prev).count());
          t_prev = t_now;
        }
        if (read_scalar(pool_full, s)) grow_pool();
        if (read_scalar(err, s)) break;
        if (rounds > (1 << 23)) throw Error(TS_ERR_INTERNAL, "saddle-saddle reduction did not converge");
      }
    }
    R->rounds_d1 = rounds;
    // (the loop ends on a host read of the active count: the stage is done)
    ctx->tuner.report(tune_key, tune_idx,
                      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_reduce).count());
    if (rstats) {
      unsigned long long h[16];
      TS_HIP(hipMemcpy(h, rstats, sizeof(h), hipMemcpyDeviceToHost));
      int wclk = 0;  // kHz
      TS_HIP(hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, ctx->device));
      const double us = wclk > 0 ? 1e3 / wclk : 0.0;
      std::fprintf(stderr,
                   "[topsimp] d1 workgroup reduction phases (us, all long columns): decision %.0f, "
                   "owner load %.0f, merge %.0f, update %.0f\n",
                   h[8] * us, h[9] * us, h[10] * us, h[11] * us);
      std::fprintf(stderr,
                   "[topsimp] d1 reduction work: lane columns %llu additions %llu; wave columns %llu "
                   "additions %llu max chain %llu; long columns %llu additions %llu max chain %llu\n",
                   h[6], h[7], h[0], h[1], h[2], h[3], h[4], h[5]);
    }
    length_stats("reduced");
    if (std::getenv("TS_TRACE"))
      std::fprintf(stderr, "[topsimp] d1 reduction: %d rounds, pool %lld / %lld words, %d grows\n",
                   rounds, (long long)read_scalar(pool.top, s), (long long)pool_cap, grows);
    k_d1_pairs<<<blocks_for(ncols), 256, 0, s>>>(col_desc, ncols, cols, pool.data, R->cid[1],
                                                 R->ckey[1], R->cid[2], R->ckey[2], po);
    ctx->timer.stop();
  }
  {
    const int h_err = read_scalar(err, s);
    if (h_err) throw Error(TS_ERR_INTERNAL, "persistence error " + std::to_string(h_err));
  }

  // ---- essential class and counts ----
  int64_t np = int64_t(read_scalar(po.count, s));
  if (np + nf > pcap) throw Error(TS_ERR_INTERNAL, "pair buffer overflow");
  if (batch) {
    unsigned int* fmin = ws.get<unsigned int>("pm.fmin", nf);
    unsigned int* fmax = ws.get<unsigned int>("pm.fmax", nf);
    k_fill_u32<<<blocks_for(nf), 256, 0, s>>>(fmin, nf, 0xFFFFFFFFu);
    k_fill_u32<<<blocks_for(nf), 256, 0, s>>>(fmax, nf, 0u);
    k_field_extrema<<<blocks_for(n, 256 * kAppendPer), 256, 0, s>>>(R->rank, GB, fmin, fmax);
    k_essential<<<blocks_for(nf), 256, 0, s>>>(fmin, fmax, R->order, nf, po, np);
    TS_HIP(hipGetLastError());
    np += nf;
  } else {
    const int32_t dim0 = 0, death = -1;
    int32_t gmin;
    TS_HIP(hipMemcpyAsync(&gmin, R->cid[0], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    const uint64_t bk = 0, dk = uint64_t(n - 1) << 12;
    TS_HIP(hipMemcpyAsync(po.dim + np, &dim0, 4, hipMemcpyHostToDevice, s));
    TS_HIP(hipMemcpyAsync(po.birth + np, &gmin, 4, hipMemcpyHostToDevice, s));
    TS_HIP(hipMemcpyAsync(po.death + np, &death, 4, hipMemcpyHostToDevice, s));
    TS_HIP(hipMemcpyAsync(po.bkey + np, &bk, 8, hipMemcpyHostToDevice, s));
    TS_HIP(hipMemcpyAsync(po.dkey + np, &dk, 8, hipMemcpyHostToDevice, s));
    TS_HIP(hipStreamSynchronize(s));
    ++np;
  }
  if (np - nf != nmin - nf + nmax + (ne - (nmin - nf)))
    throw Error(TS_ERR_INTERNAL, "pair count does not match the critical cells");
  R->npairs = np;
  R->pdim = po.dim;
  R->pbirth = po.birth;
  R->pdeath = po.death;
  R->pbkey = po.bkey;
  R->pdkey = po.dkey;

  if (std::getenv("TS_TRACE"))
    std::fprintf(stderr,
                 "[topsimp] n=%d crit=%lld/%lld/%lld/%lld rounds d0=%d d2=%d d1=%d cols=%lld\n", n,
                 (long long)nmin, (long long)ne, (long long)ntri, (long long)nmax, R->rounds_d0,
                 R->rounds_d2, R->rounds_d1, (long long)ncols);

  // ---- K8: diagram order ----
  ctx->timer.start("K8 diagram");
  uint64_t* dkeys = ws.get<uint64_t>("pm.dkeys", np);
  R->diag = ws.get<uint32_t>("pm.diag", np);
  unsigned int* nd = ws.get<unsigned int>("pm.nd", 1);
  TS_HIP(hipMemsetAsync(nd, 0, sizeof(unsigned int), s));
  k_diag_keys<<<blocks_for(np), 256, 0, s>>>(po.dim, po.bkey, po.dkey, np, dkeys, R->diag, nd);
  R->ndiag = read_scalar(nd, s);
  radix_sort_u64(ws, dkeys, R->diag, R->ndiag, 0, 64, s);
  ctx->timer.stop();
  TS_HIP(hipGetLastError());
  R->complete = true;
  if (trace) {
    TS_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "[topsimp] persistence map wall %.3f ms\n",
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                           t_wall).count());
  }
}

namespace {
__global__ void k_records(const uint32_t* __restrict__ sel, int64_t nsel, int use_sel,
                          const int32_t* __restrict__ pdim, const int32_t* __restrict__ pbirth,
                          const int32_t* __restrict__ pdeath, const uint64_t* __restrict__ bkey,
                          const uint64_t* __restrict__ dkey, const int32_t* __restrict__ order,
                          const float* __restrict__ f, ts_pair* __restrict__ out) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nsel) return;
  const uint32_t i = use_sel ? sel[k] : uint32_t(k);
  ts_pair p;
  p.dim = pdim[i];
  p.essential = pdeath[i] < 0 ? 1 : 0;
  p.birth_cell = pbirth[i];
  p.death_cell = pdeath[i];
  p.v_birth = order[bkey[i] >> 12];
  p.v_death = order[dkey[i] >> 12];
  p.birth = f[p.v_birth];
  p.death = f[p.v_death];
  out[k] = p;
}
}  // namespace

void pair_records(ts_ctx* ctx, const PersistenceResult& R, const float* f, bool diagram_only,
                  ts_pair* out_dev) {
  const int64_t n = diagram_only ? R.ndiag : R.npairs;
  if (n == 0) return;
  k_records<<<blocks_for(n), 256, 0, ctx->stream>>>(R.diag, n, diagram_only ? 1 : 0, R.pdim,
                                                    R.pbirth, R.pdeath, R.pbkey, R.pdkey, R.order,
                                                    f, out_dev);
  TS_HIP(hipGetLastError());
}

namespace {

// field of each record (by its birth vertex) as a sort key, the record index
// as the payload
__global__ void k_record_fields(const ts_pair* __restrict__ rec, int64_t n,
                                const int64_t* __restrict__ base, int nf,
                                uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = rec[i].v_birth;
  int lo = 0, hi = nf - 1;  // the last field whose base is <= v
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  key[i] = uint32_t(lo);
  val[i] = uint32_t(i);
}

// first position of each field in the sorted keys
__global__ void k_field_starts(const uint32_t* __restrict__ key, int64_t n,
                               int64_t* __restrict__ start) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0 || key[i] != key[i - 1]) start[key[i]] = i;
}

// records in field order with field-local ids (a cell id of dimension d is
// a multiple of the vertex id space: 1, 7, 12, 6 cells per anchor vertex)
__global__ void k_local_records(const ts_pair* __restrict__ rec, const uint32_t* __restrict__ key,
                                const uint32_t* __restrict__ val, int64_t n,
                                const int64_t* __restrict__ base, ts_pair* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ts_pair r = rec[val[i]];
  const int64_t b = base[key[i]];
  const int64_t per[4] = {1, 7, 12, 6};
  r.v_birth -= b;
  r.v_death -= b;
  r.birth_cell -= per[r.dim] * b;
  if (r.death_cell >= 0) r.death_cell -= per[r.dim + 1] * b;
  out[i] = r;
}

}  // namespace

void batch_diagram_records(ts_ctx* ctx, const PersistenceResult& R, const float* f,
                           const Batch& B, ts_pair* out_dev, int64_t* counts) {
  hipStream_t s = ctx->stream;
  Workspace& ws = ctx->ws;
  const int nf = int(B.grids.size());
  const int64_t n = R.ndiag;
  ts_pair* rec = ws.get<ts_pair>("bd.records", n + 1);
  pair_records(ctx, R, f, true, rec);
  int64_t* dbase = ws.get<int64_t>("bd.base", nf + 1);
  uint32_t* key = ws.get<uint32_t>("bd.key", n + 1);
  uint32_t* val = ws.get<uint32_t>("bd.val", n + 1);
  int64_t* start = ws.get<int64_t>("bd.start", nf + 1);
  TS_HIP(hipMemcpyAsync(dbase, B.base.data(), size_t(nf) * 8, hipMemcpyHostToDevice, s));
  k_fill_u64<<<blocks_for(nf + 1), 256, 0, s>>>(reinterpret_cast<uint64_t*>(start), nf + 1,
                                               uint64_t(n));
  if (n > 0) {
    k_record_fields<<<blocks_for(n), 256, 0, s>>>(rec, n, dbase, nf, key, val);
    int bits = 0;
    while ((int64_t(1) << bits) < nf) ++bits;
    radix_sort_u32(ws, key, val, size_t(n), 0, std::max(bits, 1), s);  // stable
    k_field_starts<<<blocks_for(n), 256, 0, s>>>(key, n, start);
    k_local_records<<<blocks_for(n), 256, 0, s>>>(rec, key, val, n, dbase, out_dev);
  }
  TS_HIP(hipGetLastError());
  std::vector<int64_t> h(nf + 1);
  TS_HIP(hipMemcpyAsync(h.data(), start, size_t(nf + 1) * 8, hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  h[nf] = n;
  // every field has at least its essential class, so every start is written
  for (int i = 0; i < nf; ++i) counts[i] = h[i + 1] - h[i];
}

void decode_gradient(ts_ctx* ctx, const PersistenceResult& R, int32_t* vup, int32_t* eup,
                     int32_t* tup) {
  hipStream_t s = ctx->stream;
  const NbOff off = make_offsets(R.g);
  k_valid_cells<<<blocks_for(R.g.n), 256, 0, s>>>(R.g, eup, tup);
  k_decode<<<blocks_for(R.g.n), 256, 0, s>>>(R.g, off, R.rank, R.code, vup, eup, tup);
  TS_HIP(hipGetLastError());
}

}  // namespace ts
