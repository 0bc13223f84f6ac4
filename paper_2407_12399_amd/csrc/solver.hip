// solver.hip -- the simplification loop around the persistence map.
//
// Per iteration j (Alg. 1):
//   1. gradient step on the device (Sec. 4.1): every diagram point pulls its
//      birth and death vertices towards its target; contributions are summed
//      per vertex in diagram order (one thread per vertex after a sort by
//      (vertex, kind, diagram index)), in FP32 without contraction;
//   2. persistence map of the new field (persistence.hip);
//   3. still pairs (Sec. 4.3): points with the same (dim, v_birth, v_death)
//      as a point of the previous diagram keep its assignment; the others are
//      assigned exactly, per dimension, to the targets no still point holds
//      (host: shortest augmenting paths for small problems, an auction with
//      an optimality certificate for large ones).
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <queue>
#include <sched.h>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "persistence.h"
#include "solver.h"

namespace ts {
namespace {

inline unsigned nblk(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

// diagram points in diagram order
__global__ void k_points(const uint32_t* __restrict__ diag, int64_t nd,
                         const int32_t* __restrict__ pdim, const int32_t* __restrict__ pbirth,
                         const int32_t* __restrict__ pdeath, const uint64_t* __restrict__ bkey,
                         const uint64_t* __restrict__ dkey, const int32_t* __restrict__ order,
                         const float* __restrict__ x, int32_t* __restrict__ out_i32,
                         float* __restrict__ out_f) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  const uint32_t i = diag[k];
  const int vb = order[bkey[i] >> 12], vd = order[dkey[i] >> 12];
  out_i32[6 * k + 0] = pdim[i];
  out_i32[6 * k + 1] = pdeath[i] < 0 ? 1 : 0;
  out_i32[6 * k + 2] = vb;
  out_i32[6 * k + 3] = vd;
  out_i32[6 * k + 4] = pbirth[i];
  out_i32[6 * k + 5] = pdeath[i];
  out_f[2 * k + 0] = x[vb];
  out_f[2 * k + 1] = x[vd];
}

// still-join keys (Sec. 4.3): dim << 50 | v_b << 25 | v_d, with the diagram
// index as payload (a stable sort keeps equal keys in diagram order)
__global__ void k_join_keys(const int32_t* __restrict__ pts, int64_t np, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ idx) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= np) return;
  keys[k] = (uint64_t(uint32_t(pts[6 * k])) << 50) | (uint64_t(uint32_t(pts[6 * k + 2])) << 25) |
            uint64_t(uint32_t(pts[6 * k + 3]));
  idx[k] = uint32_t(k);
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* a, int64_t n, uint64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// prev_of[i] = the previous diagram's point with the same key and the same
// occurrence rank among equal keys (the multiset join), or -1
__global__ void k_join(const uint64_t* __restrict__ ck, const uint32_t* __restrict__ ci, int64_t nc,
                       const uint64_t* __restrict__ pk, const uint32_t* __restrict__ pi, int64_t np,
                       int32_t* __restrict__ prev_of) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= nc) return;
  const uint64_t key = ck[s];
  const int64_t r = s - lower_bound_u64(ck, nc, key);
  const int64_t t = lower_bound_u64(pk, np, key) + r;
  prev_of[ci[s]] = (t < np && pk[t] == key) ? int32_t(pi[t]) : -1;
}

// contribution keys: vertex << 33 | kind << 32 | diagram index
__global__ void k_step_keys(const int32_t* __restrict__ vb, const int32_t* __restrict__ vd,
                            int64_t np, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= np) return;
  keys[2 * k] = (uint64_t(uint32_t(vb[k])) << 33) | uint64_t(k);
  keys[2 * k + 1] = (uint64_t(uint32_t(vd[k])) << 33) | (1ull << 32) | uint64_t(k);
  vals[2 * k] = uint32_t(2 * k);
  vals[2 * k + 1] = uint32_t(2 * k + 1);
}

// x[v] <- x[v] - (alpha_b * B(v) + alpha_d * D(v)), sums in diagram order
__global__ void k_step_apply(const uint64_t* __restrict__ keys, int64_t ne,
                             const float* __restrict__ tb, const float* __restrict__ td,
                             float* __restrict__ x, float alpha_b, float alpha_d,
                             uint8_t* __restrict__ changed) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const uint32_t v = uint32_t(keys[e] >> 33);
  if (e > 0 && uint32_t(keys[e - 1] >> 33) == v) return;  // not the head of its vertex
  const float xv = x[v];
  float B = 0.0f, D = 0.0f;
  for (int64_t j = e; j < ne && uint32_t(keys[j] >> 33) == v; ++j) {
    const uint32_t k = uint32_t(keys[j] & 0xFFFFFFFFull);
    if ((keys[j] >> 32) & 1ull)
      D = __fadd_rn(D, __fmul_rn(2.0f, __fsub_rn(xv, td[k])));
    else
      B = __fadd_rn(B, __fmul_rn(2.0f, __fsub_rn(xv, tb[k])));
  }
  const float s = __fadd_rn(__fmul_rn(alpha_b, B), __fmul_rn(alpha_d, D));
  float nx = __fsub_rn(xv, s);
  if (nx == 0.0f) nx = 0.0f;  // -0 -> +0
  x[v] = nx;
  // a value that compares equal keeps its place in the vertex order
  if (nx != xv) changed[v] = 1;
}

__global__ void k_minmax(const float* __restrict__ f, int64_t n, float* __restrict__ out) {
  __shared__ float smin[256], smax[256];
  float mn = INFINITY, mx = -INFINITY;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    mn = fminf(mn, f[i]);
    mx = fmaxf(mx, f[i]);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = smin[0];
    out[2 * blockIdx.x + 1] = smax[0];
  }
}

// ---------------------------------------------------------------- host side

struct Pt {
  int dim, ess;
  int vb, vd;
  int bcell, dcell;
  float b, d;
};

struct Tgt {
  int dim, ess;
  int vb0, vd0;
  float b, d;
};

double sqr(double a) { return a * a; }
double diag_cost(double b, double d) { return sqr(d - b) / 2.0; }
double pair_cost(double pb, double pd, double qb, double qd) { return sqr(pb - qb) + sqr(pd - qd); }

uint64_t pkey(int dim, int vb, int vd) {
  return (uint64_t(uint32_t(dim)) << 60) | (uint64_t(uint32_t(vb)) << 30) | uint64_t(uint32_t(vd));
}

// Interchangeable items (equal (dim, v_b, v_d) points, equal (dim, v_b0,
// v_d0) targets) receive a canonical assignment: point classes in diagram
// order take their target classes sorted by lowest member id (diagonal
// last); a target class hands out its ids in increasing order.
void canonical_classes(const std::vector<Pt>& P, const std::vector<int>& red,
                       const std::vector<Tgt>& T, std::vector<int>* phi);

// std::sort of a large vector of distinct keys on several host threads:
// sorted chunks, merged pairwise (the keys are distinct, so the result is the
// serial sort's).
template <class T>
void sort_parallel(std::vector<T>& v) {
  const size_t n = v.size();
  const int nt = int(std::min<size_t>(8, std::max<size_t>(1, n >> 16)));
  if (nt < 2) {
    std::sort(v.begin(), v.end());
    return;
  }
  std::vector<size_t> cut(size_t(nt) + 1);
  for (int t = 0; t <= nt; ++t) cut[t] = n * size_t(t) / size_t(nt);
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t] { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1]); });
    for (std::thread& x : th) x.join();
  }
  for (size_t w = 1; w < size_t(nt); w *= 2) {  // merge runs of w chunks pairwise
    std::vector<std::thread> th;
    for (size_t a = 0; a + w < size_t(nt); a += 2 * w) {
      const size_t lo = cut[a], mid = cut[a + w], hi = cut[std::min(a + 2 * w, size_t(nt))];
      th.emplace_back([&v, lo, mid, hi] {
        std::inplace_merge(v.begin() + lo, v.begin() + mid, v.begin() + hi);
      });
    }
    for (std::thread& x : th) x.join();
  }
}

// Only points in a class of two or more, or matched into a target class of
// two or more, can change; the others are left out of the class bookkeeping.
void canonical_form(const std::vector<Pt>& P, const std::vector<int>& red, const std::vector<Tgt>& T,
                    std::vector<int>* phi) {
  auto multi = [](std::vector<std::pair<uint64_t, int>>& v) {  // members of classes of >= 2
    sort_parallel(v);  // (key, point) pairs are distinct
    std::vector<int> idx;
    for (size_t a = 0; a < v.size();) {
      size_t b = a + 1;
      while (b < v.size() && v[b].first == v[a].first) ++b;
      if (b - a >= 2)
        for (size_t c = a; c < b; ++c) idx.push_back(v[c].second);
      a = b;
    }
    return idx;
  };
  std::vector<std::pair<uint64_t, int>> pk, tk;
  pk.reserve(red.size());
  for (int i : red) pk.push_back({pkey(P[i].dim, P[i].vb, P[i].vd), i});
  for (int i : red)
    if ((*phi)[i] >= 0) {
      const Tgt& t = T[(*phi)[i]];
      tk.push_back({pkey(t.dim, t.vb0, t.vd0), i});
    }
  std::vector<char> involved(P.size(), 0);
  for (int i : multi(pk)) involved[i] = 1;
  for (int i : multi(tk)) involved[i] = 1;
  std::vector<int> sub;
  for (int i : red)
    if (involved[i]) sub.push_back(i);
  if (!sub.empty()) canonical_classes(P, sub, T, phi);
}

void canonical_classes(const std::vector<Pt>& P, const std::vector<int>& red,
                       const std::vector<Tgt>& T, std::vector<int>* phi) {
  std::unordered_map<uint64_t, int> pcls_of;
  std::vector<std::vector<int>> pcls;
  for (int i : red) {
    const uint64_t k = pkey(P[i].dim, P[i].vb, P[i].vd);
    auto it = pcls_of.find(k);
    if (it == pcls_of.end()) {
      pcls_of.emplace(k, int(pcls.size()));
      pcls.push_back({i});
    } else {
      pcls[it->second].push_back(i);
    }
  }
  std::unordered_map<uint64_t, int> tcls_of;
  std::vector<std::vector<int>> tcls;
  std::vector<int> tcls_idx(T.size(), -1);
  for (int i : red) {
    const int t = (*phi)[i];
    if (t < 0) continue;
    const uint64_t k = pkey(T[t].dim, T[t].vb0, T[t].vd0);
    auto it = tcls_of.find(k);
    int c;
    if (it == tcls_of.end()) {
      c = int(tcls.size());
      tcls_of.emplace(k, c);
      tcls.push_back({});
    } else {
      c = it->second;
    }
    tcls[c].push_back(t);
    tcls_idx[t] = c;
  }
  for (auto& v : tcls) std::sort(v.begin(), v.end());
  std::vector<size_t> next(tcls.size(), 0);
  // point classes are visited in diagram order (red is in diagram order and
  // classes were created at their first member)
  for (const auto& members : pcls) {
    std::vector<std::pair<int64_t, int>> got;  // (lowest id of the class or +inf, class)
    for (int i : members) {
      const int t = (*phi)[i];
      if (t < 0) got.push_back({std::numeric_limits<int64_t>::max(), -1});
      else got.push_back({tcls[tcls_idx[t]].front(), tcls_idx[t]});
    }
    std::sort(got.begin(), got.end());
    for (size_t s = 0; s < members.size(); ++s) {
      const int c = got[s].second;
      (*phi)[members[s]] = c < 0 ? -1 : tcls[c][next[c]++];
    }
  }
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Signal selection (Sec. 3).  Threshold mode: a finite pair is non-signal
// iff its dimension is in the mask and its persistence is below
// threshold_rel * range(f0) (or equal to it, unless ties count as signal).
// List mode: a finite pair is signal iff the list holds its
// (dim, birth cell, death cell), looked up in a sorted copy of the list.  The
// essential pair is always signal.
struct SignalRule {
  const ts_signal& sig;
  double thr;
  std::vector<std::array<int64_t, 3>> listed;
  SignalRule(const ts_signal& s, double range) : sig(s), thr(double(s.threshold_rel) * range) {
    if (sig.mode == 1) {
      listed.reserve(size_t(std::max<int64_t>(sig.n_signal, 0)));
      for (int64_t q = 0; q < sig.n_signal; ++q)
        listed.push_back({int64_t(sig.signal[q].dim), sig.signal[q].birth_cell,
                          sig.signal[q].death_cell});
      std::sort(listed.begin(), listed.end());
    }
  }
  bool signal(const Pt& p) const {
    if (p.ess) return true;
    if (sig.mode == 1)
      return std::binary_search(listed.begin(), listed.end(),
                                std::array<int64_t, 3>{int64_t(p.dim), int64_t(p.bcell),
                                                       int64_t(p.dcell)});
    const double pers = double(p.d) - double(p.b);
    const bool masked = (sig.nonsignal_dim_mask >> p.dim) & 1u;
    const bool below = pers < thr || (pers == thr && !sig.ties_signal);
    return !(masked && below);
  }
};

struct Solver {
  std::vector<Tgt> T;
  int ess_target = -1;
  double gap = 0;  // assignment precision (0: exact / tight auction)

  // D_T = D(f0) minus the non-signal pairs (Sec. 3).
  void targets(const std::vector<Pt>& P0, const ts_signal& sig, double range,
               std::vector<int>* phi) {
    phi->assign(P0.size(), -1);
    const SignalRule rule(sig, range);
    for (size_t i = 0; i < P0.size(); ++i) {
      const Pt& p = P0[i];
      if (rule.signal(p)) {
        if (p.ess) ess_target = int(T.size());
        (*phi)[i] = int(T.size());
        T.push_back({p.dim, p.ess, p.vb, p.vd, p.b, p.d});
      }
    }
  }

  double loss(const std::vector<Pt>& P, const std::vector<int>& phi) const {
    double L = 0;
    for (size_t i = 0; i < P.size(); ++i)
      L += phi[i] >= 0 ? pair_cost(P[i].b, P[i].d, T[phi[i]].b, T[phi[i]].d)
                       : diag_cost(P[i].b, P[i].d);
    return L;
  }

  double max_diag_pers(const std::vector<Pt>& P, const std::vector<int>& phi) const {
    double m = 0;
    for (size_t i = 0; i < P.size(); ++i)
      if (phi[i] < 0) m = std::max(m, double(P[i].d) - double(P[i].b));
    return m;
  }

  // prev_of[i]: the still partner of point i in the previous diagram (-1 if
  // none), from the device-side join
  void assign(const std::vector<Pt>& P, const std::vector<int>& prev_of, const std::vector<int>& phip,
              std::vector<int>* phi, int64_t* n_still, int64_t* n_red) {
    const double t_join = now_s();
    phi->assign(P.size(), -1);
    std::vector<char> still(P.size(), 0), held(T.size(), 0);
    *n_still = 0;
    for (size_t i = 0; i < P.size(); ++i) {
      const int j = prev_of[i];
      if (j < 0) continue;
      still[i] = 1;
      ++*n_still;
      (*phi)[i] = phip[j];
      if ((*phi)[i] >= 0) held[(*phi)[i]] = 1;
    }
    std::vector<int> red;
    for (size_t i = 0; i < P.size(); ++i) {
      if (P[i].ess) {
        if (!still[i]) (*phi)[i] = ess_target;
        continue;
      }
      if (!still[i]) red.push_back(int(i));
    }
    *n_red = int64_t(red.size());
    const double t_build = now_s();
    // one reduced problem per dimension; the three are independent and are
    // solved on separate host threads
    struct Problem {
      std::vector<int> pi, tj, match;
      std::vector<double> pb, pd, qb, qd;
      double gap = 0;
      double seconds = 0;
      std::string error;
    };
    Problem pr[3];
    for (int dim = 0; dim < 3; ++dim) {
      Problem& q = pr[dim];
      q.gap = gap;
      for (int i : red)
        if (P[i].dim == dim) {
          q.pi.push_back(i);
          q.pb.push_back(P[i].b);
          q.pd.push_back(P[i].d);
        }
      if (q.pi.empty()) continue;
      for (size_t j = 0; j < T.size(); ++j)
        if (!held[j] && !T[j].ess && T[j].dim == dim) {
          q.tj.push_back(int(j));
          q.qb.push_back(T[j].b);
          q.qd.push_back(T[j].d);
        }
      if (const char* dir = std::getenv("TS_DUMP_ASSIGN")) {
        static int seq = 0;
        const std::string path = std::string(dir) + "/assign_" + std::to_string(seq++) + "_d" +
                                 std::to_string(dim) + ".bin";
        if (FILE* fp = std::fopen(path.c_str(), "wb")) {
          const int64_t mm = int64_t(q.pb.size()), kk = int64_t(q.qb.size());
          std::fwrite(&mm, 8, 1, fp);
          std::fwrite(&kk, 8, 1, fp);
          std::fwrite(q.pb.data(), 8, mm, fp);
          std::fwrite(q.pd.data(), 8, mm, fp);
          std::fwrite(q.qb.data(), 8, kk, fp);
          std::fwrite(q.qd.data(), 8, kk, fp);
          std::fwrite(q.tj.data(), 4, kk, fp);
          std::fclose(fp);
        }
      }
    }
    const double t_solve = now_s();
    auto solve = [](Problem* q) {
      try {
        const double t0 = now_s();
        assign_reduced(q->pb, q->pd, q->qb, q->qd, &q->match, q->gap);
        q->seconds = now_s() - t0;
      } catch (const std::exception& e) {
        q->error = e.what();
      }
    };
    std::vector<std::thread> workers;
    for (int dim = 1; dim < 3; ++dim)
      if (!pr[dim].pi.empty()) workers.emplace_back(solve, &pr[dim]);
    if (!pr[0].pi.empty()) solve(&pr[0]);
    for (std::thread& w : workers) w.join();
    for (int dim = 0; dim < 3; ++dim) {
      const Problem& q = pr[dim];
      if (q.pi.empty()) continue;
      if (!q.error.empty()) throw Error(TS_ERR_INTERNAL, q.error);
      if (std::getenv("TS_TRACE"))
        std::fprintf(stderr, "[topsimp] assign dim %d: %zu points, %zu targets, %.3f s\n", dim,
                     q.pb.size(), q.qb.size(), q.seconds);
      for (size_t s = 0; s < q.pi.size(); ++s)
        (*phi)[q.pi[s]] = q.match[s] >= 0 ? q.tj[q.match[s]] : -1;
    }
    const double t_canon = now_s();
    canonical_form(P, red, T, phi);
    if (std::getenv("TS_TRACE"))
      std::fprintf(stderr,
                   "[topsimp] assign host: still join %.3f s, problems %.3f s, solve %.3f s, "
                   "canonical form %.3f s\n",
                   t_build - t_join, t_solve - t_build, t_canon - t_solve, now_s() - t_canon);
  }
};

template <class T>
T* dev(ts_ctx* ctx, const char* name, size_t n) {
  return ctx->ws.get<T>(name, n);
}

void fetch_points(ts_ctx* ctx, const PersistenceResult& R, const float* x, std::vector<Pt>* P) {
  hipStream_t s = ctx->stream;
  const int64_t nd = R.ndiag;
  int32_t* di = dev<int32_t>(ctx, "sim.pi", 6 * nd + 6);
  float* df = dev<float>(ctx, "sim.pf", 2 * nd + 2);
  k_points<<<nblk(nd), 256, 0, s>>>(R.diag, nd, R.pdim, R.pbirth, R.pdeath, R.pbkey, R.pdkey,
                                    R.order, x, di, df);
  TS_HIP(hipGetLastError());
  std::vector<int32_t> hi(6 * nd);
  std::vector<float> hf(2 * nd);
  TS_HIP(hipMemcpyAsync(hi.data(), di, hi.size() * 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipMemcpyAsync(hf.data(), df, hf.size() * 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  P->resize(nd);
  for (int64_t k = 0; k < nd; ++k) {
    Pt& p = (*P)[k];
    p.dim = hi[6 * k];
    p.ess = hi[6 * k + 1];
    p.vb = hi[6 * k + 2];
    p.vd = hi[6 * k + 3];
    p.bcell = hi[6 * k + 4];
    p.dcell = hi[6 * k + 5];
    p.b = hf[2 * k];
    p.d = hf[2 * k + 1];
  }
}


}  // namespace

// ---------------------------------------------------------------- assignment

namespace {

// Values |p - q_u|^2 - s_u of one KD-tree leaf's members (coordinates and
// scores contiguous; a masked member has score -inf and value +inf), and the
// bit mask of the members whose value is <= thr.  Built
// for AVX-512, AVX2 and baseline x86-64, picked at load time by the CPU; the
// same IEEE operations in the same order in every variant (no contraction),
// so all give the same values bit for bit.
#if defined(__HIP_DEVICE_COMPILE__)
#define TS_HOST_CLONES
#else
#define TS_HOST_CLONES __attribute__((target_clones("avx512f", "avx2", "default")))
#endif
TS_HOST_CLONES uint64_t leaf_values(const double* __restrict__ x, const double* __restrict__ y,
                                    const double* __restrict__ s, int cnt, double px, double py,
                                    double thr, double* __restrict__ out) {
  for (int u = 0; u < cnt; ++u) {
    const double dx = x[u] - px, dy = y[u] - py;
    out[u] = (dx * dx + dy * dy) - s[u];
  }
  uint64_t m = 0;
  for (int u = 0; u < cnt; ++u) m |= uint64_t(out[u] <= thr) << u;
  return m;
}

// Largest of a leaf's scores (-inf if all are masked): max is exact, so the
// four running maxima of the vector form give the scalar loop's result.
TS_HOST_CLONES double leaf_max(const double* __restrict__ s, int cnt) {
  double m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  int u = 0;
  for (; u + 4 <= cnt; u += 4)
    for (int l = 0; l < 4; ++l) m[l] = m[l] < s[u + l] ? s[u + l] : m[l];
  for (; u < cnt; ++u) m[0] = m[0] < s[u] ? s[u] : m[0];
  const double a = m[0] < m[1] ? m[1] : m[0], b = m[2] < m[3] ? m[3] : m[2];
  return a < b ? b : a;
}

// 2D KD-tree over the targets (birth, death).  Every target j carries a
// score s_j (or "masked"); a node keeps the largest unmasked score below it.
// best(p) returns the unmasked target minimising |p - q_j|^2 - s_j.  Leaf
// members are stored contiguously in tree order (coordinates, score, mask,
// id), so that a leaf scan reads one short run of memory.
struct KDTree {
  struct Node {
    double x0, x1, y0, y1, smax;
    int left, right, parent, begin, end;
  };
  std::vector<Node> nodes;
  std::vector<int> idx, leaf_of, pos_of;
  std::vector<double> s;     // score by target id
  std::vector<char> masked;  // mask by target id
  std::vector<double> lx, ly, ls;  // coordinates and score (-inf if masked) in tree order
  const double* X = nullptr;
  const double* Y = nullptr;
  static constexpr double NEG = -std::numeric_limits<double>::infinity();
  // Targets per leaf.  The queries return the same answer for any tree shape
  // (a node's bound never exceeds the value of a target below it, in floating
  // point too, since every step of both is monotone), so this only sets the
  // balance between node visits and leaf scans: on the auction's problems 32
  // is about 12 % faster than 8, and 16 or 64 are no faster than 32.
  static constexpr int kLeaf = 64;

  void build(const double* x, const double* y, int k) {
    X = x;
    Y = y;
    idx.resize(k);
    for (int j = 0; j < k; ++j) idx[j] = j;
    leaf_of.assign(k, -1);
    s.assign(k, 0.0);
    masked.assign(k, 0);
    nodes.clear();
    if (k > 0) make(0, k, -1);
    pos_of.assign(k, -1);
    lx.resize(k);
    ly.resize(k);
    ls.assign(k, 0.0);
    for (int t = 0; t < k; ++t) {
      pos_of[idx[t]] = t;
      lx[t] = X[idx[t]];
      ly[t] = Y[idx[t]];
    }
  }
  int make(int b, int e, int parent) {
    Node nd;
    nd.x0 = nd.y0 = std::numeric_limits<double>::infinity();
    nd.x1 = nd.y1 = -std::numeric_limits<double>::infinity();
    for (int i = b; i < e; ++i) {
      nd.x0 = std::min(nd.x0, X[idx[i]]);
      nd.x1 = std::max(nd.x1, X[idx[i]]);
      nd.y0 = std::min(nd.y0, Y[idx[i]]);
      nd.y1 = std::max(nd.y1, Y[idx[i]]);
    }
    nd.begin = b;
    nd.end = e;
    nd.left = nd.right = -1;
    nd.parent = parent;
    nd.smax = NEG;
    const int id = int(nodes.size());
    nodes.push_back(nd);
    if (e - b > kLeaf) {
      const int mid = (b + e) / 2;
      const bool byx = (nd.x1 - nd.x0) >= (nd.y1 - nd.y0);
      std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int a, int c) {
        return byx ? (X[a] < X[c] || (X[a] == X[c] && a < c))
                   : (Y[a] < Y[c] || (Y[a] == Y[c] && a < c));
      });
      const int l = make(b, mid, id);
      const int r = make(mid, e, id);
      nodes[id].left = l;
      nodes[id].right = r;
    } else {
      for (int i = b; i < e; ++i) leaf_of[idx[i]] = id;
    }
    return id;
  }
  void set_all(const std::vector<double>& sc) {
    s = sc;
    std::fill(masked.begin(), masked.end(), 0);
    for (size_t t = 0; t < idx.size(); ++t) ls[t] = s[idx[t]];
    for (int i = int(nodes.size()) - 1; i >= 0; --i) refresh(i);
  }
  void refresh(int id) {
    Node& nd = nodes[id];
    if (nd.left < 0) {
      nd.smax = leaf_max(&ls[nd.begin], nd.end - nd.begin);
    } else {
      nd.smax = std::max(nodes[nd.left].smax, nodes[nd.right].smax);
    }
  }
  // change target j (score / mask) and the maxima above it
  void update(int j, double sj, bool mask) {
    const double old = masked[j] ? NEG : s[j];  // j's contribution to the maxima
    const double now = mask ? NEG : sj;
    s[j] = sj;
    masked[j] = mask;
    ls[pos_of[j]] = now;
    const int leaf = leaf_of[j];
    if (now >= old) {  // the maxima on the path can only rise, to `now`
      for (int id = leaf; id >= 0 && nodes[id].smax < now; id = nodes[id].parent) nodes[id].smax = now;
      return;
    }
    if (old < nodes[leaf].smax) return;  // j was not a maximiser: nothing changes
    for (int id = leaf; id >= 0; id = nodes[id].parent) {
      const double before = nodes[id].smax;
      refresh(id);
      if (nodes[id].smax == before && id != leaf) break;
    }
  }
  static double d2box(const Node& nd, double px, double py) {
    const double dx = px < nd.x0 ? nd.x0 - px : (px > nd.x1 ? px - nd.x1 : 0.0);
    const double dy = py < nd.y0 ? nd.y0 - py : (py > nd.y1 ? py - nd.y1 : 0.0);
    return dx * dx + dy * dy;
  }
  // the two smallest values of |p - q_j|^2 - s_j over unmasked j (depth
  // first, nearer child first, pruned by the node bounds); the result does
  // not depend on the visiting order: v1 is the minimum, the returned id the
  // lowest id attaining it, v2 the second smallest value of the multiset.
  // hint[0..1]: two target ids (or -1) counted before the descent, so that
  // the pruning starts from their values (a caller passes the previous
  // answer of the same point); on return, the best id and an id attaining v2.
  int best2(double px, double py, double* v1, double* v2, int* hint) const {
    *v1 = *v2 = std::numeric_limits<double>::infinity();
    int bj = -1, j2 = -1;
    const int h0 = hint[0], h1 = hint[1] != hint[0] ? hint[1] : -1;
    hint[0] = hint[1] = -1;
    if (nodes.empty() || nodes[0].smax == NEG) return -1;
    auto offer = [&](double v, int j) {
      if (v < *v1 || (v == *v1 && j < bj)) {
        *v2 = *v1;
        j2 = bj;
        *v1 = v;
        bj = j;
      } else if (v < *v2) {
        *v2 = v;
        j2 = j;
      }
    };
    for (const int h : {h0, h1})
      if (h >= 0 && !masked[h]) {
        const int t = pos_of[h];
        const double dx = lx[t] - px, dy = ly[t] - py;
        offer((dx * dx + dy * dy) - ls[t], h);
      }
    // depth-first stack: it grows by at most one entry per tree level (the
    // median splits keep the depth below 26 for any int-sized target set)
    double sb[64];
    int sn[64];
    int top_n = 0;
    sb[0] = d2box(nodes[0], px, py) - nodes[0].smax;
    sn[0] = 0;
    top_n = 1;
    while (top_n > 0) {
      --top_n;
      const std::pair<double, int> top = {sb[top_n], sn[top_n]};
      if (top.first > *v2) continue;
      const Node& nd = nodes[top.second];
      if (nd.left < 0) {
        // values of the whole leaf first (vector code), then the running
        // two smallest among those not above the second smallest so far
        // (which only falls during the scan)
        double vals[kLeaf];
        const int cnt = nd.end - nd.begin;
        uint64_t m = leaf_values(&lx[nd.begin], &ly[nd.begin], &ls[nd.begin], cnt, px, py, *v2, vals);
        while (m) {
          const int u = __builtin_ctzll(m);
          m &= m - 1;
          const double v = vals[u];
          if (!(v <= *v2)) continue;
          const int j = idx[nd.begin + u];
          if (j != h0 && j != h1) offer(v, j);  // the hints are counted already
        }
      } else {
        const Node& L = nodes[nd.left];
        const Node& R = nodes[nd.right];
        const double bl = L.smax == NEG ? INFINITY : d2box(L, px, py) - L.smax;
        const double br = R.smax == NEG ? INFINITY : d2box(R, px, py) - R.smax;
        // push the farther child first so that the nearer one is visited first
        if (bl <= br) {
          if (br <= *v2) { sb[top_n] = br; sn[top_n++] = nd.right; }
          if (bl <= *v2) { sb[top_n] = bl; sn[top_n++] = nd.left; }
        } else {
          if (bl <= *v2) { sb[top_n] = bl; sn[top_n++] = nd.left; }
          if (br <= *v2) { sb[top_n] = br; sn[top_n++] = nd.right; }
        }
      }
    }
    hint[0] = bj;
    hint[1] = j2;
    return bj;
  }
  // Every unmasked j with |p - q_j|^2 - s_j < thr, appended to out (nodes
  // whose bound d2box - smax is already >= thr are skipped).
  void collect(double px, double py, double thr, std::vector<int>* out) const {
    if (nodes.empty() || nodes[0].smax == NEG) return;
    int sn[64];
    int top_n = 0;
    sn[top_n++] = 0;
    while (top_n > 0) {
      const Node& nd = nodes[sn[--top_n]];
      if (nd.smax == NEG || !(d2box(nd, px, py) - nd.smax < thr)) continue;
      if (nd.left < 0) {
        for (int t = nd.begin; t < nd.end; ++t) {
          if (ls[t] == NEG) continue;  // masked
          const double dx = lx[t] - px, dy = ly[t] - py;
          if ((dx * dx + dy * dy) - ls[t] < thr) out->push_back(idx[t]);
        }
      } else {
        sn[top_n++] = nd.left;
        sn[top_n++] = nd.right;
      }
    }
  }
  // argmin over unmasked j of |p - q_j|^2 - s_j; ties to the lower index.
  // seed (or -1): a target counted before the descent, so that the search
  // starts from its value (same answer).
  int best(double px, double py, double* val, int seed = -1) const {
    *val = std::numeric_limits<double>::infinity();
    int bj = -1;
    if (nodes.empty() || nodes[0].smax == NEG) return -1;
    if (seed >= 0 && !masked[seed]) {
      const int t = pos_of[seed];
      const double dx = lx[t] - px, dy = ly[t] - py;
      *val = (dx * dx + dy * dy) - ls[t];
      bj = seed;
    }
    typedef std::pair<double, int> NI;  // (lower bound, node)
    std::priority_queue<NI, std::vector<NI>, std::greater<NI>> todo;
    todo.push({d2box(nodes[0], px, py) - nodes[0].smax, 0});
    while (!todo.empty()) {
      const NI top = todo.top();
      todo.pop();
      if (top.first > *val) break;
      const Node& nd = nodes[top.second];
      if (nd.left < 0) {
        for (int t = nd.begin; t < nd.end; ++t) {
          if (ls[t] == NEG) continue;  // masked
          const double dx = lx[t] - px, dy = ly[t] - py;
          const double v = (dx * dx + dy * dy) - ls[t];
          if (v < *val || (v == *val && idx[t] < bj)) {
            *val = v;
            bj = idx[t];
          }
        }
      } else {
        for (int c : {nd.left, nd.right})
          if (nodes[c].smax != NEG) todo.push({d2box(nodes[c], px, py) - nodes[c].smax, c});
      }
    }
    return bj;
  }
};

// Optimality certificate for an assignment of the square augmented problem
// (min-cost form).  Persons are the points 0..m-1 and one diagonal copy per
// target (m + j); objects are the targets 0..k-1 and one diagonal copy per
// point (k + i).  Point i may take any target j at c(p_i, q_j) or its own
// copy at diag(p_i); target copy m + j may take target j at diag(q_j) or any
// point copy at 0.  With object prices p, an assignment is optimal when every
// person x holding o_x attains the minimum over its objects of cost(x, o) +
// p_o (complementary slackness with the feasible duals u_x = that minimum,
// v_o = -p_o).  An epsilon-scaled auction leaves every person within eps of
// its minimum.  The check lowers the price of a person's object until the
// person attains its minimum, p_o = min - cost(x, o): a label-correcting
// shortest-path computation over the fixed assignment, in which the object
// whose price fell can become the strict minimum of other persons, who are
// checked in turn.  When no person is left above its minimum the assignment
// is optimal.  If it is not, prices keep falling around a cycle of persons
// who would all gain by trading objects: every lowering records the object
// that set the new price, and a cycle among those records has negative total
// cost (Bellman-Ford predecessor graphs), so the persons on it trade along
// it, which lowers the total cost, and the checks go on.  A person counts as
// above its minimum only by more than 4 ulps of the terms of the two values
// compared (|cost| + |price| of its object and of the minimising one), the
// size of their rounding: with prices of either sign a sum can cancel far
// below its terms.
struct Certificate {
  int64_t lowerings = 0, trades = 0;
  bool ok = false;
};

struct CertificateMissing {};

Certificate certify_assignment(const std::vector<double>& pb, const std::vector<double>& pd,
                               const std::vector<double>& qb, const std::vector<double>& qd,
                               const std::vector<double>& dp, const std::vector<double>& dq,
                               std::vector<double>* price_io, std::vector<int>* holds_io) {
  const int m = int(pb.size()), k = int(qb.size());
  const int NP = m + k;
  std::vector<double>& price = *price_io;
  std::vector<int>& holds = *holds_io;
  std::vector<int> owner(k + m, -1);
  for (int x = 0; x < NP; ++x) owner[holds[x]] = x;
  const double INF = std::numeric_limits<double>::infinity();
  auto cost = [&](int x, int o) {
    if (x < m) return o < k ? pair_cost(pb[x], pd[x], qb[o], qd[o]) : (o == k + x ? dp[x] : INF);
    const int j = x - m;
    return o < k ? (o == j ? dq[j] : INF) : 0.0;
  };
  auto slack_tol = [&](int x, int o, int arg) {
    const double a = std::fabs(cost(x, o)) + std::fabs(price[o]);
    const double b = arg >= 0 ? std::fabs(cost(x, arg)) + std::fabs(price[arg]) : 0.0;
    return 4.0 * std::numeric_limits<double>::epsilon() * std::max(a, b) + 1e-300;
  };
  std::vector<double> lam(NP);
  for (int x = 0; x < NP; ++x) lam[x] = cost(x, holds[x]) + price[holds[x]];
  double scale = 0;  // cost scale: largest diagonal costs
  for (double v : dp) scale = std::max(scale, v);
  for (double v : dq) scale = std::max(scale, v);
  // targets by (c + price): s_j = -p_j
  KDTree tt;
  tt.build(qb.data(), qd.data(), k);
  {
    std::vector<double> sc(k);
    for (int j = 0; j < k; ++j) sc[j] = -price[j];
    tt.set_all(sc);
  }
  // points by their current value lam_i, for the reverse question "which
  // points now prefer target j"
  KDTree pt;
  pt.build(pb.data(), pd.data(), m);
  pt.set_all(std::vector<double>(lam.begin(), lam.begin() + m));
  // lowest point-copy price (lazy min-heap) and target copies by lam (lazy max-heap)
  typedef std::pair<double, int> DI;
  std::priority_queue<DI, std::vector<DI>, std::greater<DI>> cheap;
  for (int i = 0; i < m; ++i) cheap.push({price[k + i], i});
  auto min_copy = [&](int* who) {
    while (!cheap.empty() && cheap.top().first != price[k + cheap.top().second]) cheap.pop();
    if (cheap.empty()) {
      *who = -1;
      return INF;
    }
    *who = k + cheap.top().second;
    return cheap.top().first;
  };
  std::priority_queue<DI> tcl;
  for (int j = 0; j < k; ++j) tcl.push({lam[m + j], m + j});
  std::vector<int> queue;
  std::vector<char> inq(NP, 1);
  queue.reserve(NP);
  for (int x = 0; x < NP; ++x) queue.push_back(x);
  std::vector<int> from(k + m, -1), count(k + m, 0), seen(k + m, -1);
  std::vector<int> hits;
  std::vector<int> hint(2 * size_t(std::max(m, 1)), -1);
  Certificate cert;
  const int64_t budget = int64_t(64) * NP + 100000;
  int walk = 0;
  auto push = [&](int y) {
    if (!inq[y]) {
      inq[y] = 1;
      queue.push_back(y);
    }
  };
  // the exact minimum of person x and the object attaining it
  auto minimum = [&](int x, int* arg) {
    if (x < m) {
      double v1, v2;
      int j = tt.best2(pb[x], pd[x], &v1, &v2, &hint[2 * size_t(x)]);
      double best = INF;
      *arg = -1;
      if (j >= 0) {
        best = v1;
        *arg = j;
      }
      const double vd = dp[x] + price[k + x];
      if (vd < best) {
        best = vd;
        *arg = k + x;
      }
      return best;
    }
    const int j = x - m;
    int c;
    const double pc = min_copy(&c);
    const double vt = dq[j] + price[j];
    if (pc < vt) {
      *arg = c;
      return pc;
    }
    *arg = j;
    return vt;
  };
  auto set_lam = [&](int x) {
    lam[x] = cost(x, holds[x]) + price[holds[x]];
    if (x < m) pt.update(x, lam[x], false);
    else tcl.push({lam[x], x});
  };
  // objects whose price fell: who else may now prefer them
  auto after_lowering = [&](int o) {
    if (o < k) {
      tt.update(o, -price[o], false);
      hits.clear();
      // superset by a small margin; every hit is checked exactly
      const double thr = -price[o] + 1e-12 * (std::fabs(price[o]) + scale);
      pt.collect(qb[o], qd[o], thr, &hits);
      for (int i : hits) push(i);
      push(m + o);
    } else {
      const int i = o - k;
      cheap.push({price[o], i});
      push(i);
      while (!tcl.empty()) {
        const DI top = tcl.top();
        if (top.first != lam[top.second] || inq[top.second]) {
          tcl.pop();
          continue;
        }
        if (!(top.first > price[o])) break;
        tcl.pop();
        push(top.second);
      }
    }
  };
  size_t head = 0;
  while (head < queue.size()) {
    const int x = queue[head++];
    inq[x] = 0;
    if (head > (size_t(1) << 22) && head * 2 > queue.size()) {  // compact the queue
      queue.erase(queue.begin(), queue.begin() + head);
      head = 0;
    }
    int arg;
    const double mu = minimum(x, &arg);
    if (x >= m) tcl.push({lam[x], x});  // keep it findable by lam
    const int o = holds[x];
    if (!(mu < lam[x] - slack_tol(x, o, arg))) continue;
    if (arg == o) continue;  // cannot happen with exact minima; be safe
    price[o] = mu - cost(x, o);
    from[o] = arg;
    set_lam(x);
    after_lowering(o);
    if (++cert.lowerings > budget) return cert;
    if (++count[o] % 8 != 0) continue;
    // look for a cycle among the recorded objects, starting from o
    ++walk;
    int cur = o;
    while (cur >= 0 && seen[cur] != walk) {
      seen[cur] = walk;
      cur = from[cur];
    }
    if (cur < 0) continue;
    // cur lies on a cycle: trade along it if it really saves cost
    std::vector<int> cyc;
    int c = cur;
    do {
      cyc.push_back(c);
      c = from[c];
    } while (c != cur && int(cyc.size()) <= k + m);
    if (c != cur) continue;
    double gain = 0;
    for (size_t t = 0; t < cyc.size(); ++t) {
      const int ob = cyc[t], nb = cyc[(t + 1) % cyc.size()];
      gain += cost(owner[ob], nb) - cost(owner[ob], ob);
    }
    if (!(gain < 0) || !std::isfinite(gain)) continue;
    std::vector<int> who(cyc.size());
    for (size_t t = 0; t < cyc.size(); ++t) who[t] = owner[cyc[t]];
    for (size_t t = 0; t < cyc.size(); ++t) {
      const int nb = cyc[(t + 1) % cyc.size()];
      holds[who[t]] = nb;
      owner[nb] = who[t];
    }
    for (size_t t = 0; t < cyc.size(); ++t) {
      from[cyc[t]] = -1;
      set_lam(who[t]);
      push(who[t]);
    }
    ++cert.trades;
  }
  cert.ok = true;
  return cert;
}

}  // namespace

// The searches of a window of queued bidders: for b < n, the two best items
// of tree for the query (qx[id], qy[id]), id = ids[b], started from the
// bidder's hints (read, not written: the caller keeps them in out[b]).
struct Found {
  int j, h0, h1;  // best item, and the hints the search leaves (best, second)
  double c1, c2;  // smallest and second smallest values
};
struct SearchJob {
  const KDTree* tree;
  const double* qx;
  const double* qy;
  const int* ids;
  const int* hints;
  Found* out;
  void operator()(int b) const {
    const int id = ids[b];
    Found& F = out[b];
    int h[2] = {hints[2 * size_t(id)], hints[2 * size_t(id) + 1]};
    F.j = tree->best2(qx[id], qy[id], &F.c1, &F.c2, h);
    F.h0 = h[0];
    F.h1 = h[1];
  }
};

// Host threads that run a window's searches at once.  run(job, n) spreads
// job(0..n-1) over the workers and the calling thread and returns when all
// are done; the searches only read shared state.  Workers spin between
// windows (they come microseconds apart during an auction) and yield after a
// while.  Extra threads come from a process-wide budget (several auctions run
// at once: the dimensions of a field, the fields of a batch), so that the
// host is not oversubscribed; a pool that gets no thread runs everything on
// the caller.
class WindowPool {
 public:
  explicit WindowPool(int want) {
    int got = 0;
    for (int have = budget().load(); want > 0 && have > 0;) {
      const int take = std::min(want, have);
      if (budget().compare_exchange_weak(have, have - take)) {
        got = take;
        break;
      }
    }
    for (int t = 0; t < got; ++t) th_.emplace_back([this] { loop(); });
  }
  ~WindowPool() {
    stop_.store(true, std::memory_order_release);
    gen_.fetch_add(1, std::memory_order_acq_rel);
    for (std::thread& t : th_) t.join();
    budget().fetch_add(int(th_.size()));
  }
  int threads() const { return int(th_.size()) + 1; }
  // threads an auction asks for: half the budget (two large auctions, those
  // of dimensions 0 and 2, usually run at once)
  static int share() {
    static const int s = std::max(1, budget().load() / 2);
    return s;
  }
  void run(const SearchJob& job, int n) {
    job_ = job;
    n_ = n;
    next_.store(0, std::memory_order_relaxed);
    busy_.store(int(th_.size()), std::memory_order_relaxed);
    gen_.fetch_add(1, std::memory_order_acq_rel);
    work();
    while (busy_.load(std::memory_order_acquire) > 0) pause();
  }

 private:
  // threads beyond one per running auction: TS_ASSIGN_THREADS, else the CPUs
  // this process may run on (at most 16) less two
  static std::atomic<int>& budget() {
    static std::atomic<int> b{[] {
      if (const char* e = std::getenv("TS_ASSIGN_THREADS")) return std::max(0, std::atoi(e));
      cpu_set_t set;
      int cpus = 1;
      if (sched_getaffinity(0, sizeof(set), &set) == 0) cpus = CPU_COUNT(&set);
      return std::max(0, std::min(cpus, 16) - 2);
    }()};
    return b;
  }
  static void pause() { __builtin_ia32_pause(); }
  void work() {
    for (int i; (i = next_.fetch_add(1, std::memory_order_relaxed)) < n_;) job_(i);
  }
  void loop() {
    int seen = 0;
    for (;;) {
      int g;
      for (int spins = 0; (g = gen_.load(std::memory_order_acquire)) == seen;)
        if (++spins < 20000) pause();
        else std::this_thread::yield();
      seen = g;
      if (stop_.load(std::memory_order_acquire)) return;
      work();
      busy_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  std::vector<std::thread> th_;
  std::atomic<int> gen_{0}, next_{0}, busy_{0};
  std::atomic<bool> stop_{false};
  SearchJob job_{};
  int n_ = 0;
};

// Auction on the rectangular form of the problem.  Sending every target to
// the diagonal costs sum diag(q); from there, point p pays
// c'(p,q) = c(p,q) - diag(q) for taking target q (at most one point per
// target) or diag(p) for its own diagonal.  Persons are the points, objects
// the targets (prices pi_q >= 0) and each point's private diagonal (no
// price).  Complementary slackness asks every point to hold a cheapest
// option (cost plus price) and every target nobody holds to have price 0.
// Forward bids (Bertsekas) raise the price of a point's best target by the gap
// to its second best option plus eps.  Prices carry over between the phases of
// epsilon scaling, so a target may end a phase with no holder and a positive
// price: it then makes reverse bids, offering itself to the point that gains
// most from it at the price the second such point would pay (less eps), or
// dropping to price 0 when no point gains more than eps.  Forward bids end
// with every point within eps of its cheapest option, reverse bids keep that
// and end with every unheld target at price 0.  Bids use KD-trees over the
// targets (score diag(q) - pi_q) and over the points (score: what each pays).
// In exact mode (gap_rel == 0) the final state, written as one of the square
// augmented problem, is then certified optimal (certify_assignment); with
// gap_rel > 0 the phases stop once the assignment's total is within
// (1 + gap_rel)^2 of the dual lower bound, with no certificate.
double assign_auction(const std::vector<double>& pb, const std::vector<double>& pd,
                      const std::vector<double>& qb, const std::vector<double>& qd,
                      std::vector<int>* match, double eps_rel, double gap_rel) {
  const int m = int(pb.size()), k = int(qb.size());
  match->assign(m, -1);
  std::vector<double> dp(m), dq(k);
  double maxdp = 0, maxdq = 0;
  for (int i = 0; i < m; ++i) maxdp = std::max(maxdp, dp[i] = diag_cost(pb[i], pd[i]));
  for (int j = 0; j < k; ++j) maxdq = std::max(maxdq, dq[j] = diag_cost(qb[j], qd[j]));
  const double W = std::max(maxdp + maxdq, 1e-300);
  const bool trace = std::getenv("TS_TRACE") != nullptr;
  std::vector<double> pi(dq);     // target prices, started at diag(q)
  std::vector<int> owner(k, -1);  // target -> point
  std::vector<int> holds(m, -1);  // point -> target, or k for its diagonal
  std::vector<double> pay(m, 0.0);  // what each point pays for its holding
  KDTree tt;
  tt.build(qb.data(), qd.data(), k);
  tt.set_all(std::vector<double>(k, 0.0));  // diag(q) - pi_q
  KDTree pt;
  pt.build(pb.data(), pd.data(), m);
  std::vector<int> hints(2 * size_t(std::max(m, 1)), -1), rhints(2 * size_t(std::max(k, 1)), -1);
  auto cprime = [&](int i, int j) { return pair_cost(pb[i], pd[i], qb[j], qd[j]) - dq[j]; };
  // Windows of queued bidders search at once against the state before the
  // window (read-only), then commit in queue order as the serial auction
  // would.  Within a phase, forward bids only raise target prices and reverse
  // bids only lower what points pay, so every search value can only grow
  // while a window commits: a result whose best and second-best items were
  // not changed by an earlier commit of the window is the serial search's
  // result (the same minimum, lowest id attaining it, and second value); any
  // other is searched again at its turn.  The bids, prices and matching are
  // those of the serial auction.
  constexpr int kWindow = 128, kMinWindow = 4;
  auto pool_owner = std::make_unique<WindowPool>(m + k >= 4096 ? WindowPool::share() : 0);
  WindowPool& pool = *pool_owner;
  std::vector<Found> found(kWindow);
  std::vector<int> ttouch(k, 0), ptouch(m, 0);  // window stamp of the last change
  int stamp = 0;
  auto set_price = [&](int j, double v) {
    pi[j] = v;
    ttouch[j] = stamp;
    tt.update(j, dq[j] - v, false);
  };
  double eps = W / 4.0;
  const double eps_final = W * eps_rel;
  const int64_t bid_cap = int64_t(400) * (m + k) + 1000000;
  std::vector<int> queue, rqueue;
  for (int phase = 0;; ++phase) {
    std::fill(owner.begin(), owner.end(), -1);
    std::fill(holds.begin(), holds.end(), -1);
    queue.clear();
    for (int i = 0; i < m; ++i) queue.push_back(i);
    int64_t fbids = 0, rbids = 0, redone = 0, nwin = 0;
    double twin = 0;
    const double tphase = now_s();
    size_t wbeg = 0, wend = 0;  // the current window of searched bidders
    for (size_t head = 0; head < queue.size(); ++head) {
      if (head >= wend && pool.threads() > 1 && queue.size() - head >= size_t(kMinWindow)) {
        wbeg = head;
        wend = head + std::min(queue.size() - head, size_t(kWindow));
        ++stamp;
        const double tw = now_s();
        pool.run({&tt, pb.data(), pd.data(), &queue[head], hints.data(), found.data()},
                 int(wend - head));
        twin += now_s() - tw;
        ++nwin;
      }
      const int i = queue[head];
      double c1, c2;  // the two smallest c' + pi over the targets
      int j;
      const Found* F = head < wend ? &found[head - wbeg] : nullptr;
      if (F && (F->h0 < 0 || ttouch[F->h0] != stamp) && (F->h1 < 0 || ttouch[F->h1] != stamp)) {
        j = F->j;
        c1 = F->c1;
        c2 = F->c2;
        hints[2 * size_t(i)] = F->h0;
        hints[2 * size_t(i) + 1] = F->h1;
      } else {
        if (F) ++redone;
        j = tt.best2(pb[i], pd[i], &c1, &c2, &hints[2 * size_t(i)]);
      }
      if (++fbids > bid_cap) throw Error(TS_ERR_INTERNAL, "assignment: auction did not settle");
      if (j < 0 || dp[i] <= c1) {  // its diagonal (ties go to the diagonal)
        holds[i] = k;
        pay[i] = dp[i];
        continue;
      }
      set_price(j, pi[j] + (std::min(c2, dp[i]) - c1) + eps);
      const int prev = owner[j];
      owner[j] = i;
      holds[i] = j;
      pay[i] = cprime(i, j) + pi[j];
      if (prev >= 0) {
        holds[prev] = -1;
        queue.push_back(prev);
      }
    }
    rqueue.clear();
    for (int j = 0; j < k; ++j)
      if (owner[j] < 0 && pi[j] > 0) rqueue.push_back(j);
    if (!rqueue.empty()) {
      pt.set_all(pay);
      size_t wbeg = 0, wend = 0;
      for (size_t head = 0; head < rqueue.size(); ++head) {
        if (head >= wend && pool.threads() > 1 && rqueue.size() - head >= size_t(kMinWindow)) {
          wbeg = head;
          wend = head + std::min(rqueue.size() - head, size_t(kWindow));
          ++stamp;
          const double tw = now_s();
          pool.run({&pt, qb.data(), qd.data(), &rqueue[head], rhints.data(), found.data()},
                   int(wend - head));
          twin += now_s() - tw;
          ++nwin;
        }
        const int j = rqueue[head];
        if (owner[j] >= 0 || !(pi[j] > 0)) continue;
        if (++rbids > bid_cap) throw Error(TS_ERR_INTERNAL, "assignment: auction did not settle");
        double v1, v2;  // the two smallest |p - q|^2 - pay_p over the points
        int i1;
        const Found* F = head < wend ? &found[head - wbeg] : nullptr;
        if (F && (F->h0 < 0 || ptouch[F->h0] != stamp) && (F->h1 < 0 || ptouch[F->h1] != stamp)) {
          i1 = F->j;
          v1 = F->c1;
          v2 = F->c2;
          rhints[2 * size_t(j)] = F->h0;
          rhints[2 * size_t(j) + 1] = F->h1;
        } else {
          if (F) ++redone;
          i1 = pt.best2(qb[j], qd[j], &v1, &v2, &rhints[2 * size_t(j)]);
        }
        const double g1 = dq[j] - v1, g2 = dq[j] - v2;  // pay_p - c'(p, q)
        if (i1 < 0 || g1 <= eps) {
          set_price(j, 0.0);
          continue;
        }
        set_price(j, std::max(0.0, std::min(pi[j], g2 - eps)));
        const int old = holds[i1];
        owner[j] = i1;
        holds[i1] = j;
        pay[i1] = cprime(i1, j) + pi[j];
        ptouch[i1] = stamp;
        pt.update(i1, pay[i1], false);
        if (old < k) {
          owner[old] = -1;
          if (pi[old] > 0) rqueue.push_back(old);
        }
      }
    }
    if (trace)
      std::fprintf(stderr,
                   "[topsimp] auction phase %d eps %.3g bids %lld forward, %lld reverse, %lld "
                   "searched again; %.3f s, %lld windows %.3f s\n",
                   phase, eps, (long long)fbids, (long long)rbids, (long long)redone,
                   now_s() - tphase, (long long)nwin, twin);
    if (eps <= eps_final) break;
    if (gap_rel > 0) {
      // dual bound: for prices pi >= 0 and u_p = the cheapest option of p,
      // every assignment costs at least sum diag(q) + sum u_p - sum pi_q
      double primal = 0, lower = 0;
      for (int j = 0; j < k; ++j) {
        lower += dq[j] - pi[j];
        if (owner[j] < 0) primal += dq[j];
      }
      for (int i = 0; i < m; ++i) {
        double val;
        const int j = tt.best(pb[i], pd[i], &val, hints[2 * size_t(i)]);
        lower += j >= 0 ? std::min(dp[i], val) : dp[i];
        primal += holds[i] < k ? pair_cost(pb[i], pd[i], qb[holds[i]], qd[holds[i]]) : dp[i];
      }
      if (trace)
        std::fprintf(stderr, "[topsimp] auction phase %d total %.9g lower bound %.9g\n", phase,
                     primal, lower);
      if (lower > 0 && primal <= (1 + gap_rel) * (1 + gap_rel) * lower) break;
    }
    eps = std::max(eps / 4.0, eps_final);  // a factor of 4 needs the fewest bids on noisy diagrams
  }
  pool_owner.reset();  // the workers are not needed after the bids
  // the state as one of the square problem: target j at price pi_j - diag(q_j)
  // and the point copies at 0, except that a point on its diagonal may pay up
  // to its margin for its own copy (that headroom keeps the certificate's
  // lowerings local); a target copy holds its target when no point does,
  // else the copy of a point that holds a target
  std::vector<int> sholds(m + k, -1);
  std::vector<double> price(k + m, 0.0);
  for (int j = 0; j < k; ++j) price[j] = pi[j] - dq[j];
  std::vector<int> spare;
  for (int i = 0; i < m; ++i) {
    if (holds[i] < k) {
      sholds[i] = holds[i];
      spare.push_back(k + i);
    } else {
      sholds[i] = k + i;
    }
  }
  for (int j = 0, s = 0; j < k; ++j) sholds[m + j] = owner[j] < 0 ? j : spare[s++];
  if (gap_rel == 0) {
    tt.set_all([&] {
      std::vector<double> sc(k);
      for (int j = 0; j < k; ++j) sc[j] = -price[j];
      return sc;
    }());
    for (int i = 0; i < m; ++i) {
      if (holds[i] < k) continue;
      double v1, v2;
      int h[2] = {-1, -1};
      if (tt.best2(pb[i], pd[i], &v1, &v2, h) >= 0 && v1 - dp[i] > 0) price[k + i] = v1 - dp[i];
    }
    const double tc = now_s();
    const Certificate c = certify_assignment(pb, pd, qb, qd, dp, dq, &price, &sholds);
    if (trace)
      std::fprintf(stderr, "[topsimp] certificate %s: %lld lowerings, %lld trades, %.3f s\n",
                   c.ok ? "ok" : "not reached", (long long)c.lowerings, (long long)c.trades,
                   now_s() - tc);
    if (!c.ok) throw CertificateMissing();
  }
  double total = 0;
  std::vector<char> used(k, 0);
  for (int i = 0; i < m; ++i) {
    const int o = sholds[i];
    if (o < k && pair_cost(pb[i], pd[i], qb[o], qd[o]) < dp[i] + dq[o]) {
      (*match)[i] = o;
      used[o] = 1;
      total += pair_cost(pb[i], pd[i], qb[o], qd[o]);
    } else {
      total += dp[i];
    }
  }
  for (int j = 0; j < k; ++j)
    if (!used[j]) total += dq[j];
  return total;
}

double assign_exact(const std::vector<double>& pb, const std::vector<double>& pd,
                    const std::vector<double>& qb, const std::vector<double>& qd,
                    std::vector<int>* match) {
  // Maximum-weight matching: a point p matched to a target q saves
  // w(p,q) = diag(p) + diag(q) - c(p,q) over sending both to the diagonal;
  // only pairs with w > 0 can be in an optimum (a pair with w <= 0 is
  // dissolved at the end: both go to the diagonal, as the pruning rule says).
  // Rows-perfect assignment of the points to the targets or to their own
  // diagonal column, with costs W - w >= 0 and W on the diagonal column,
  // solved exactly by shortest augmenting paths (Dijkstra with potentials)
  // on the complete graph: the cheapest unsettled target of a row is a
  // KD-tree query, since its reduced cost is
  //   (W - diag(p) - u_p) + |p - q|^2 - (diag(q) + v_q).
  const int m = int(pb.size()), k = int(qb.size());
  match->assign(m, -1);
  std::vector<double> dp(m), dq(k);
  double maxdp = 0, maxdq = 0;
  for (int i = 0; i < m; ++i) maxdp = std::max(maxdp, dp[i] = diag_cost(pb[i], pd[i]));
  for (int j = 0; j < k; ++j) maxdq = std::max(maxdq, dq[j] = diag_cost(qb[j], qd[j]));
  double total = 0;
  if (m == 0) {
    for (int j = 0; j < k; ++j) total += dq[j];
    return total;
  }
  const double W = maxdp + maxdq;
  const double INF = std::numeric_limits<double>::infinity();
  KDTree tree;
  tree.build(qb.data(), qd.data(), k);
  std::vector<double> v(k, 0.0), u(m, 0.0), sc(k);
  for (int j = 0; j < k; ++j) sc[j] = dq[j];
  tree.set_all(sc);
  // column ids: targets 0..k-1; the diagonal column of row r is k + r
  std::vector<int> row_of(k, -1), col_of(m, -1), way(k + m, -1);
  std::vector<double> dcol(k + m, INF), drow(m, 0.0);
  std::vector<int> settled_list, tree_rows;
  struct Cand {
    double d;
    int row, col;
    bool operator>(const Cand& o) const {
      if (d != o.d) return d > o.d;
      if (col != o.col) return col > o.col;
      return row > o.row;
    }
  };
  for (int s0 = 0; s0 < m; ++s0) {
    std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> pq;
    settled_list.clear();
    tree_rows.clear();
    auto offer_best = [&](int r) {
      double val;
      const int j = tree.best(pb[r], pd[r], &val);
      if (j >= 0) pq.push({drow[r] + (W - dp[r] - u[r]) + val, r, j});
    };
    auto enter = [&](int r, double dr) {
      drow[r] = dr;
      tree_rows.push_back(r);
      offer_best(r);
      pq.push({dr + W - u[r], r, k + r});  // its diagonal column (potential 0, always free)
    };
    enter(s0, 0.0);
    int found = -1;
    double D = 0;
    while (!pq.empty()) {
      const Cand c = pq.top();
      pq.pop();
      if (c.col >= k) {  // a row's own diagonal column is free
        found = c.col;
        D = c.d;
        way[found] = c.row;
        break;
      }
      if (tree.masked[c.col]) {  // settled meanwhile: offer the row's next best
        offer_best(c.row);
        continue;
      }
      const int j = c.col;
      dcol[j] = c.d;
      way[j] = c.row;
      tree.update(j, tree.s[j], true);
      settled_list.push_back(j);
      if (row_of[j] < 0) {
        found = j;
        D = c.d;
        break;
      }
      enter(row_of[j], c.d);
      offer_best(c.row);
    }
    if (found < 0) throw Error(TS_ERR_INTERNAL, "assignment: no augmenting path");
    for (int r : tree_rows) u[r] += D - drow[r];
    for (int j : settled_list) {
      v[j] -= D - dcol[j];
      dcol[j] = INF;
      tree.update(j, dq[j] + v[j], false);
    }
    // augment
    int j = found;
    int guard = 0;
    while (true) {
      if (++guard > k + m + 2) throw Error(TS_ERR_INTERNAL, "assignment: augmenting path loops");
      const int r = way[j];
      const int prev = col_of[r];
      col_of[r] = j;
      if (j < k) row_of[j] = r;
      if (r == s0) break;
      j = prev;
    }
  }
  std::vector<char> used(k, 0);
  for (int i = 0; i < m; ++i) {
    const int j = col_of[i];
    if (j < k && pair_cost(pb[i], pd[i], qb[j], qd[j]) < dp[i] + dq[j]) {
      (*match)[i] = j;
      used[j] = 1;
      total += pair_cost(pb[i], pd[i], qb[j], qd[j]);
    } else {
      total += dp[i];
    }
  }
  for (int j = 0; j < k; ++j)
    if (!used[j]) total += dq[j];
  return total;
}

namespace {

// Indices of the set B (KD-tree `tree` over B, scores s_b = diag(b)) that
// are among the `topk` best of some query a by saving
// w = diag(a) + diag(b) - c(a,b) > 0 (ties with the last one kept).  The
// positivity test has a relative margin, so that no candidate is lost to
// rounding.
std::vector<int> top_candidates(KDTree* tree, const std::vector<double>& ab,
                                const std::vector<double>& ad, const std::vector<double>& da,
                                double scale, int nb, int topk) {
  std::vector<char> keep(nb, 0);
  std::vector<int> masked;
  for (size_t a = 0; a < ab.size(); ++a) {
    const double bound = da[a] + 1e-9 * (da[a] + scale) + 1e-300;
    masked.clear();
    double last = 0;
    for (int t = 0;; ++t) {
      double v;
      const int b = tree->best(ab[a], ad[a], &v);
      if (b < 0 || !(v < bound)) break;
      if (t >= topk && v > last + 1e-12 * (std::fabs(last) + scale)) break;
      keep[b] = 1;
      last = v;
      tree->update(b, tree->s[b], true);
      masked.push_back(b);
    }
    for (int b : masked) tree->update(b, tree->s[b], false);
  }
  std::vector<int> out;
  for (int b = 0; b < nb; ++b)
    if (keep[b]) out.push_back(b);
  return out;
}

// Indices a of the query set with some b of the tree at a positive saving
// (same margin).  The searches of a large query set run on a WindowPool.
std::vector<int> has_candidate(const KDTree& tree, const std::vector<double>& ab,
                               const std::vector<double>& ad, const std::vector<double>& da,
                               double scale) {
  const int n = int(ab.size());
  std::vector<int> ids(n), hints(2 * size_t(n), -1);
  for (int a = 0; a < n; ++a) ids[a] = a;
  std::vector<Found> res(static_cast<size_t>(n));
  {
    WindowPool pool(n >= 4096 ? WindowPool::share() : 0);
    pool.run({&tree, ab.data(), ad.data(), ids.data(), hints.data(), res.data()}, n);
  }
  std::vector<int> out;
  for (int a = 0; a < n; ++a)
    if (res[a].j >= 0 && res[a].c1 < da[a] + 1e-9 * (da[a] + scale) + 1e-300) out.push_back(a);
  return out;
}

}  // namespace

// The solver's assignment: exact reductions first, then successive shortest
// paths up to a problem size (TS_EXACT_MAX, default 1000 points + targets)
// and the certified auction above it.  Reductions, each of which keeps every
// optimum:
//  (a) a point (target) with no target (point) at a positive saving
//      w = diag(p) + diag(q) - c(p,q) goes to the diagonal;
//  (b) with k targets left, a target is matched in an optimum to one of its
//      k best points by saving: otherwise one of those is free and takes its
//      place with a larger saving.  The same holds with the roles swapped.
double assign_reduced(const std::vector<double>& pb, const std::vector<double>& pd,
                      const std::vector<double>& qb, const std::vector<double>& qd,
                      std::vector<int>* match, double gap_rel, bool auction_only) {
  if (gap_rel > 0) auction_only = true;
  int64_t limit = auction_only ? 0 : 1000;
  if (const char* e = std::getenv("TS_EXACT_MAX"); e && !auction_only) limit = std::atoll(e);
  const int m = int(pb.size()), k = int(qb.size());
  match->assign(m, -1);
  std::vector<double> dp(m), dq(k);
  double maxdp = 0, maxdq = 0;
  for (int i = 0; i < m; ++i) maxdp = std::max(maxdp, dp[i] = diag_cost(pb[i], pd[i]));
  for (int j = 0; j < k; ++j) maxdq = std::max(maxdq, dq[j] = diag_cost(qb[j], qd[j]));
  if (m + k <= 64 && !auction_only) return assign_exact(pb, pd, qb, qd, match);

  // rows and columns still in the problem (indices into the inputs)
  std::vector<int> rows(m), cols(k);
  for (int i = 0; i < m; ++i) rows[i] = i;
  for (int j = 0; j < k; ++j) cols[j] = j;
  auto gather = [](const std::vector<double>& v, const std::vector<int>& ix) {
    std::vector<double> o(ix.size());
    for (size_t t = 0; t < ix.size(); ++t) o[t] = v[ix[t]];
    return o;
  };
  // side 0: points (rows), side 1: targets (columns)
  std::vector<int>* idx[2] = {&rows, &cols};
  const std::vector<double>* B[2] = {&pb, &qb};
  const std::vector<double>* D[2] = {&pd, &qd};
  const std::vector<double>* S[2] = {&dp, &dq};
  const double scale = maxdp + maxdq;
  auto make_tree = [&](int side, KDTree* tree, std::vector<double>* b, std::vector<double>* d) {
    *b = gather(*B[side], *idx[side]);
    *d = gather(*D[side], *idx[side]);
    tree->build(b->data(), d->data(), int(b->size()));
    tree->set_all(gather(*S[side], *idx[side]));
  };
  auto prune = [&](int side) {  // (a): items of `side` with no partner in the other side
    std::vector<int>& mine = *idx[side];
    if (mine.empty()) return;
    KDTree tree;
    std::vector<double> tb, td;
    make_tree(1 - side, &tree, &tb, &td);
    const std::vector<int> keep = has_candidate(tree, gather(*B[side], mine),
                                                gather(*D[side], mine), gather(*S[side], mine),
                                                scale);
    std::vector<int> kept(keep.size());
    for (size_t t = 0; t < keep.size(); ++t) kept[t] = mine[keep[t]];
    mine.swap(kept);
  };
  auto top_k = [&](int side) {  // (b): keep the k best of `side` of every item of the other
    std::vector<int>& mine = *idx[side];
    const std::vector<int>& other = *idx[1 - side];
    KDTree tree;
    std::vector<double> tb, td;
    make_tree(side, &tree, &tb, &td);
    const std::vector<int> keep =
        top_candidates(&tree, gather(*B[1 - side], other), gather(*D[1 - side], other),
                       gather(*S[1 - side], other), scale, int(mine.size()), int(other.size()));
    std::vector<int> kept(keep.size());
    for (size_t t = 0; t < keep.size(); ++t) kept[t] = mine[keep[t]];
    mine.swap(kept);
  };
  const double t_red = now_s();
  prune(0);
  prune(1);
  if (!cols.empty() && int64_t(rows.size()) > 4 * int64_t(cols.size()))
    top_k(0);  // few targets
  else if (!rows.empty() && int64_t(cols.size()) > 4 * int64_t(rows.size()))
    top_k(1);  // few points
  if (std::getenv("TS_TRACE"))
    std::fprintf(stderr, "[topsimp] assignment reductions: %d x %d -> %zu x %zu, %.3f s\n", m, k,
                 rows.size(), cols.size(), now_s() - t_red);

  const std::vector<double> rb = gather(pb, rows), rd = gather(pd, rows);
  const std::vector<double> cb = gather(qb, cols), cd = gather(qd, cols);
  std::vector<int> sub;
  if (int64_t(rows.size() + cols.size()) <= limit) {
    assign_exact(rb, rd, cb, cd, &sub);
  } else {
    // exact mode: the auction to eps = 1e-10 W, then the optimality
    // certificate; if the certificate's work budget runs out (many cycles
    // left), once more from a 100 times smaller eps
    const double eps0 = std::getenv("TS_AUCTION_EPS") ? std::atof(std::getenv("TS_AUCTION_EPS")) : 1e-10;
    if (gap_rel > 0) {
      assign_auction(rb, rd, cb, cd, &sub, eps0, gap_rel);
    } else {
      try {
        assign_auction(rb, rd, cb, cd, &sub, eps0, 0.0);
      } catch (const CertificateMissing&) {
        try {
          assign_auction(rb, rd, cb, cd, &sub, eps0 * 1e-2, 0.0);
        } catch (const CertificateMissing&) {
          throw Error(TS_ERR_INTERNAL, "assignment: no optimality certificate");
        }
      }
    }
  }
  std::vector<char> used(k, 0);
  for (size_t t = 0; t < rows.size(); ++t)
    if (sub[t] >= 0) {
      (*match)[rows[t]] = cols[sub[t]];
      used[cols[sub[t]]] = 1;
    }
  double total = 0;
  for (int i = 0; i < m; ++i) {
    const int j = (*match)[i];
    total += j >= 0 ? pair_cost(pb[i], pd[i], qb[j], qd[j]) : dp[i];
  }
  for (int j = 0; j < k; ++j)
    if (!used[j]) total += dq[j];
  return total;
}

// ---------------------------------------------------------------- loop

namespace {

// One field of a solve and its solver state between iterations.
struct FieldRun {
  int64_t base = 0, n = 0;  // vertex range in the (batch) field buffer
  Solver S;
  std::vector<Pt> P;  // diagram points, batch vertex and cell ids
  std::vector<int> phi;
  double range = 0, tol = 0, L0 = 0, L = 0;
  bool cancelled = false;
  int iterations = 0;
  int64_t n_still = 0, n_red = 0;
};

// The solve of one field (batch == nullptr) or of a batch of fields stored
// one after another, whose persistence maps run together (every stage one
// launch over the batch).  Each field follows its own Alg. 1: its own
// targets, still join, assignment and stop rule; a field that stops is no
// longer updated, so its result is that of a solve of the field alone.
int simplify_fields(ts_ctx* ctx, int nf, const float* const* f, const Grid& G,
                    const Batch* batch, const ts_signal& sig, const ts_options& opt,
                    float* const* g_out, ts_report* reps) {
  const double t0 = now_s();
  hipStream_t s = ctx->stream;
  const int n = G.n;
  std::vector<FieldRun> F(nf);
  std::vector<int64_t> bases(nf + 1, 0);
  for (int i = 0; i < nf; ++i) {
    F[i].base = batch ? batch->base[i] : 0;
    F[i].n = batch ? batch->grids[i].n : n;
    bases[i + 1] = F[i].base + F[i].n;
    std::memset(&reps[i], 0, sizeof(ts_report));
  }
  auto field_index = [&](int v) {
    return nf == 1 ? 0
                   : int(std::upper_bound(bases.begin(), bases.end(), int64_t(v)) - bases.begin()) - 1;
  };
  float* x = dev<float>(ctx, "sim.x", n);
  float* f0 = dev<float>(ctx, "sim.f0", n);
  uint8_t* changed = dev<uint8_t>(ctx, "sim.changed", n);
  for (int i = 0; i < nf; ++i)
    TS_HIP(hipMemcpyAsync(f0 + F[i].base, f[i], size_t(F[i].n) * 4,
                          opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  TS_HIP(hipMemcpyAsync(x, f0, size_t(n) * 4, hipMemcpyDeviceToDevice, s));

  double pers_s = 0, assign_s = 0, update_s = 0;
  int64_t n_regrad = 0;
  PersistenceResult R;
  double tp = now_s();
  compute_persistence(ctx, x, G, &R, nullptr, batch);  // also rejects non-finite values
  pers_s += now_s() - tp;

  // range of every field of f0
  {
    const int nb = 256;
    float* mm = dev<float>(ctx, "sim.mm", size_t(2) * nb * nf);
    for (int i = 0; i < nf; ++i)
      k_minmax<<<nb, 256, 0, s>>>(f0 + F[i].base, F[i].n, mm + size_t(2) * nb * i);
    std::vector<float> h(size_t(2) * nb * nf);
    TS_HIP(hipMemcpyAsync(h.data(), mm, h.size() * 4, hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nf; ++i) {
      const float* hb = h.data() + size_t(2) * nb * i;
      double mn = hb[0], mx = hb[1];
      for (int b = 0; b < nb; ++b) {
        mn = std::min(mn, double(hb[2 * b]));
        mx = std::max(mx, double(hb[2 * b + 1]));
      }
      F[i].range = mx - mn;
      F[i].tol = double(opt.cancel_tol_rel) * F[i].range;
    }
  }

  // points of the batch diagram, split per field (each field's points stay in
  // its own diagram order); local[k] = index of batch point k in its field
  auto split = [&](const std::vector<Pt>& all, std::vector<std::vector<Pt>>* per,
                   std::vector<std::vector<int64_t>>* gidx, std::vector<int32_t>* local) {
    per->assign(nf, {});
    gidx->assign(nf, {});
    local->resize(all.size());
    for (size_t k = 0; k < all.size(); ++k) {
      const int i = field_index(all[k].vb);
      (*local)[k] = int32_t((*per)[i].size());
      (*per)[i].push_back(all[k]);
      (*gidx)[i].push_back(int64_t(k));
    }
  };
  std::vector<Pt> P;
  fetch_points(ctx, R, x, &P);
  int slot = 0;
  int64_t nkeys[2] = {0, 0};
  auto sort_keys = [&](int sl, int64_t np) {
    const std::string tag = std::to_string(sl);
    uint64_t* k = dev<uint64_t>(ctx, ("sim.jk" + tag).c_str(), np + 1);
    uint32_t* ix = dev<uint32_t>(ctx, ("sim.ji" + tag).c_str(), np + 1);
    if (np > 0) {
      k_join_keys<<<nblk(np), 256, 0, s>>>(dev<int32_t>(ctx, "sim.pi", 6 * np + 6), np, k, ix);
      radix_sort_u64(ctx->ws, k, ix, size_t(np), 0, 52, s);
    }
    nkeys[sl] = np;
  };
  std::vector<std::vector<Pt>> per;
  std::vector<std::vector<int64_t>> gidx;
  std::vector<int32_t> local_prev;
  split(P, &per, &gidx, &local_prev);
  auto done = [&](const FieldRun& r, double Lc) {
    if (opt.stop_mode == 1) return Lc <= double(opt.loss_ratio_s) * r.L0;
    return r.S.max_diag_pers(r.P, r.phi) < r.tol;
  };
  for (int i = 0; i < nf; ++i) {
    FieldRun& r = F[i];
    r.P.swap(per[i]);
    r.S.gap = double(opt.assign_precision);
    r.S.targets(r.P, sig, r.range, &r.phi);
    r.L0 = r.L = r.S.loss(r.P, r.phi);
    r.n_still = int64_t(r.P.size());
  }
  // still join on the device: each diagram's keys sorted once, in diagram
  // order within equal keys (slots alternate between iterations)
  sort_keys(slot, int64_t(P.size()));
  auto join = [&](int64_t nc, std::vector<int>* prev_of) {
    prev_of->assign(nc, -1);
    const int prev = slot;
    slot ^= 1;
    sort_keys(slot, nc);
    const std::string c = std::to_string(slot), q = std::to_string(prev);
    int32_t* po = dev<int32_t>(ctx, "sim.prev_of", nc + 1);
    if (nc > 0) {
      k_join<<<nblk(nc), 256, 0, s>>>(dev<uint64_t>(ctx, ("sim.jk" + c).c_str(), nc + 1),
                                      dev<uint32_t>(ctx, ("sim.ji" + c).c_str(), nc + 1), nc,
                                      dev<uint64_t>(ctx, ("sim.jk" + q).c_str(), nkeys[prev] + 1),
                                      dev<uint32_t>(ctx, ("sim.ji" + q).c_str(), nkeys[prev] + 1),
                                      nkeys[prev], po);
      TS_HIP(hipGetLastError());
      TS_HIP(hipMemcpyAsync(prev_of->data(), po, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    TS_HIP(hipStreamSynchronize(s));
  };
  // a given start field (one field): its diagram is joined with D(f0) and
  // assigned like an iteration's; it replaces f0 only if its loss is no higher
  int init_used = 0;
  if (opt.init && nf == 1) {
    FieldRun& r = F[0];
    TS_HIP(hipMemcpyAsync(x, opt.init, size_t(n) * 4,
                          opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    tp = now_s();
    compute_persistence(ctx, x, G, &R);
    std::vector<Pt> Pw;
    fetch_points(ctx, R, x, &Pw);
    pers_s += now_s() - tp;
    const double ta = now_s();
    std::vector<int> pof, phiw;
    join(int64_t(Pw.size()), &pof);
    int64_t ns = 0, nr = 0;
    r.S.assign(Pw, pof, r.phi, &phiw, &ns, &nr);
    const double Lw = r.S.loss(Pw, phiw);
    assign_s += now_s() - ta;
    if (Lw <= r.L0) {
      init_used = 1;
      r.P = Pw;
      r.phi.swap(phiw);
      r.L = Lw;
      r.n_still = ns;
      r.n_red = nr;
      P.swap(Pw);
    } else {  // back to f0 (the map and the join keys must describe the current field)
      TS_HIP(hipMemcpyAsync(x, f0, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
      tp = now_s();
      compute_persistence(ctx, x, G, &R);
      fetch_points(ctx, R, x, &P);
      pers_s += now_s() - tp;
      slot ^= 1;
      sort_keys(slot, int64_t(P.size()));
    }
    split(P, &per, &gidx, &local_prev);
  }
  int n_active = 0;
  for (FieldRun& r : F) {
    r.cancelled = opt.stop_mode == 0 && done(r, r.L);
    n_active += r.cancelled ? 0 : 1;
  }
  // per-iteration trace of a single-field solve
  auto trace = [&](int jj) {
    if (!opt.trace || nf != 1 || jj >= opt.trace_cap) return;
    double* t = opt.trace + 4 * size_t(jj);
    t[0] = now_s() - t0;
    t[1] = F[0].L;
    t[2] = F[0].S.max_diag_pers(F[0].P, F[0].phi);
    t[3] = assign_s;
  };
  trace(0);
  int j = 0;
  while (n_active > 0 && j < opt.j_max) {
    ++j;
    // ---- gradient step of the fields still running ----
    const double tu = now_s();
    {
      std::vector<int32_t> hvb, hvd;
      std::vector<float> htb, htd;
      for (const FieldRun& r : F) {
        if (r.cancelled) continue;
        for (size_t k = 0; k < r.P.size(); ++k) {
          hvb.push_back(r.P[k].vb);
          hvd.push_back(r.P[k].vd);
          if (r.phi[k] >= 0) {
            htb.push_back(r.S.T[r.phi[k]].b);
            htd.push_back(r.S.T[r.phi[k]].d);
          } else {
            const float mid = (r.P[k].b + r.P[k].d) * 0.5f;
            htb.push_back(mid);
            htd.push_back(mid);
          }
        }
      }
      const int64_t np = int64_t(hvb.size());
      int32_t* dvb = dev<int32_t>(ctx, "sim.vb", np);
      int32_t* dvd = dev<int32_t>(ctx, "sim.vd", np);
      float* dtb = dev<float>(ctx, "sim.tb", np);
      float* dtd = dev<float>(ctx, "sim.td", np);
      uint64_t* keys = dev<uint64_t>(ctx, "sim.skeys", 2 * np);
      uint32_t* vals = dev<uint32_t>(ctx, "sim.svals", 2 * np);
      TS_HIP(hipMemcpyAsync(dvb, hvb.data(), np * 4, hipMemcpyHostToDevice, s));
      TS_HIP(hipMemcpyAsync(dvd, hvd.data(), np * 4, hipMemcpyHostToDevice, s));
      TS_HIP(hipMemcpyAsync(dtb, htb.data(), np * 4, hipMemcpyHostToDevice, s));
      TS_HIP(hipMemcpyAsync(dtd, htd.data(), np * 4, hipMemcpyHostToDevice, s));
      ctx->timer.start("K10 update");
      TS_HIP(hipMemsetAsync(changed, 0, size_t(n), s));
      if (np > 0) {
        k_step_keys<<<nblk(np), 256, 0, s>>>(dvb, dvd, np, keys, vals);
        const int vbits = 33 + 32 - __builtin_clz(uint32_t(std::max(n - 1, 1)));
        radix_sort_u64(ctx->ws, keys, vals, size_t(2 * np), 0, vbits, s);
        k_step_apply<<<nblk(2 * np), 256, 0, s>>>(keys, 2 * np, dtb, dtd, x, opt.alpha_b,
                                                  opt.alpha_d, changed);
      }
      ctx->timer.stop();
      TS_HIP(hipGetLastError());
      TS_HIP(hipStreamSynchronize(s));
    }
    update_s += now_s() - tu;
    // ---- persistence ----
    tp = now_s();
    compute_persistence(ctx, x, G, &R, opt.full_gradient ? nullptr : changed, batch);
    n_regrad += R.n_regrad;
    std::vector<Pt> Pn;
    fetch_points(ctx, R, x, &Pn);
    pers_s += now_s() - tp;
    // ---- still join (whole batch) and assignment (per field) ----
    const double ta = now_s();
    std::vector<int> prev_of;
    join(int64_t(Pn.size()), &prev_of);
    std::vector<int32_t> local_n;
    split(Pn, &per, &gidx, &local_n);
    // a still partner is a point of the same field (the join key holds the
    // batch vertex ids): its index in that field's previous points
    std::vector<int> todo;
    for (int i = 0; i < nf; ++i)
      if (!F[i].cancelled) todo.push_back(i);
    std::vector<std::string> errs(nf);
    auto run_field = [&](int i) {
      try {
        FieldRun& r = F[i];
        std::vector<int> pof(per[i].size(), -1);
        for (size_t k = 0; k < per[i].size(); ++k) {
          const int pg = prev_of[gidx[i][k]];
          if (pg >= 0) pof[k] = local_prev[pg];
        }
        std::vector<int> phin;
        r.S.assign(per[i], pof, r.phi, &phin, &r.n_still, &r.n_red);
        r.P.swap(per[i]);
        r.phi.swap(phin);
        r.L = r.S.loss(r.P, r.phi);
        r.iterations = j;
        r.cancelled = done(r, r.L);
      } catch (const std::exception& e) {
        errs[i] = e.what();
      }
    };
    if (todo.size() == 1) {
      run_field(todo[0]);
    } else {
      // fields on a few host threads (each solves its dimensions on threads too)
      const int nw = int(std::min<size_t>(todo.size(), 8));
      std::atomic<size_t> next{0};
      std::vector<std::thread> workers;
      for (int w = 0; w < nw; ++w)
        workers.emplace_back([&]() {
          for (size_t t = next++; t < todo.size(); t = next++) run_field(todo[t]);
        });
      for (std::thread& w : workers) w.join();
    }
    for (int i = 0; i < nf; ++i)
      if (!errs[i].empty()) throw Error(TS_ERR_INTERNAL, errs[i]);
    n_active = 0;
    for (const FieldRun& r : F) n_active += r.cancelled ? 0 : 1;
    local_prev.swap(local_n);
    assign_s += now_s() - ta;
    trace(j);
  }
  for (FieldRun& r : F)
    if (!r.cancelled) r.iterations = j;

  // ---- outputs and reports ----
  std::vector<float> hx(n), hf(n);
  TS_HIP(hipMemcpyAsync(hx.data(), x, size_t(n) * 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipMemcpyAsync(hf.data(), f0, size_t(n) * 4, hipMemcpyDeviceToHost, s));
  if (opt.inputs_on_device)
    for (int i = 0; i < nf; ++i)
      TS_HIP(hipMemcpyAsync(g_out[i], x + F[i].base, size_t(F[i].n) * 4,
                            hipMemcpyDeviceToDevice, s));
  TS_HIP(hipStreamSynchronize(s));
  bool all = true;
  for (int i = 0; i < nf; ++i) {
    const FieldRun& r = F[i];
    ts_report* rep = &reps[i];
    if (!opt.inputs_on_device) std::memcpy(g_out[i], hx.data() + r.base, size_t(r.n) * 4);
    rep->iterations = r.iterations;
    rep->cancelled = r.cancelled ? 1 : 0;
    all = all && r.cancelled;
    rep->loss0 = r.L0;
    rep->loss = r.L;
    {
      std::vector<char> used(r.S.T.size(), 0);
      for (int t : r.phi)
        if (t >= 0) used[t] = 1;
      double un = 0;
      for (size_t t = 0; t < r.S.T.size(); ++t)
        if (!used[t]) un += diag_cost(r.S.T[t].b, r.S.T[t].d);
      rep->energy = r.L + un;
    }
    double linf = 0, l2 = 0;
    for (int64_t v = r.base; v < r.base + r.n; ++v) {
      const double d = double(hx[v]) - double(hf[v]);
      linf = std::max(linf, std::fabs(d));
      l2 += d * d;
    }
    rep->linf = linf;
    rep->l2 = std::sqrt(l2);
    rep->max_nonsignal_pers = r.S.max_diag_pers(r.P, r.phi);
    double disp = 0;
    for (size_t k = 0; k < r.P.size(); ++k)
      if (r.phi[k] >= 0)
        disp = std::max(disp, std::sqrt(pair_cost(r.P[k].b, r.P[k].d, r.S.T[r.phi[k]].b,
                                                  r.S.T[r.phi[k]].d)));
    rep->max_signal_disp = disp;
    rep->range = r.range;
    for (const Pt& p : r.P)
      if (!p.ess) rep->n_pairs[p.dim]++;
    rep->n_still = r.n_still;
    rep->n_reduced = r.n_red;
    rep->n_targets = int64_t(r.S.T.size());
    // times and the gradient work are those of the whole (batch) solve
    rep->persistence_s = pers_s;
    rep->assign_s = assign_s;
    rep->update_s = update_s;
    rep->n_regradient = n_regrad;
    rep->init_used = init_used;
    rep->total_s = now_s() - t0;
  }
  return all ? TS_OK : TS_WARN_NOT_CANCELLED;
}

}  // namespace

int simplify(ts_ctx* ctx, const float* f, const Grid& G, const ts_signal& sig,
             const ts_options& opt, float* g_out, ts_report* rep) {
  return simplify_fields(ctx, 1, &f, G, nullptr, sig, opt, &g_out, rep);
}

int simplify_batch(ts_ctx* ctx, const Batch& B, const float* const* f, const ts_signal& sig,
                   const ts_options& opt, float* const* g_out, ts_report* reps) {
  const int nf = int(B.grids.size());
  const Grid G{0, 0, 0, int(B.base[nf])};
  return simplify_fields(ctx, nf, f, G, &B, sig, opt, g_out, reps);
}

int64_t signal_mask(ts_ctx* ctx, const float* f_dev, const Grid& G, const ts_signal& sig,
                    float* mask, int on_device) {
  hipStream_t s = ctx->stream;
  PersistenceResult R;
  compute_persistence(ctx, f_dev, G, &R);  // also rejects non-finite values
  std::vector<Pt> P;
  fetch_points(ctx, R, f_dev, &P);
  const int nb = 256;
  float* mm = dev<float>(ctx, "sim.mm", 2 * nb);
  k_minmax<<<nb, 256, 0, s>>>(f_dev, G.n, mm);
  TS_HIP(hipGetLastError());
  std::vector<float> h(2 * nb);
  TS_HIP(hipMemcpyAsync(h.data(), mm, h.size() * 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  double mn = h[0], mx = h[1];
  for (int b = 0; b < nb; ++b) {
    mn = std::min(mn, double(h[2 * b]));
    mx = std::max(mx, double(h[2 * b + 1]));
  }
  const SignalRule rule(sig, mx - mn);
  std::vector<float> m(G.n, 0.0f);
  int64_t count = 0;
  for (const Pt& p : P)
    if (rule.signal(p)) {
      m[p.vb] = 1.0f;
      m[p.vd] = 1.0f;
      ++count;
    }
  if (on_device) {
    TS_HIP(hipMemcpyAsync(mask, m.data(), size_t(G.n) * 4, hipMemcpyHostToDevice, s));
    TS_HIP(hipStreamSynchronize(s));
  } else {
    std::copy(m.begin(), m.end(), mask);
  }
  return count;
}

}  // namespace ts
