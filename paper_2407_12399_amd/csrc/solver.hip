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
//      (host, sparse shortest augmenting paths).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <queue>
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
                             float* __restrict__ x, float alpha_b, float alpha_d) {
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
void canonical_form(const std::vector<Pt>& P, const std::vector<int>& red, const std::vector<Tgt>& T,
                    std::vector<int>* phi) {
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

struct Solver {
  std::vector<Tgt> T;
  int ess_target = -1;

  // Signal selection (Sec. 3): D_T = D(f0) minus the non-signal pairs.
  void targets(const std::vector<Pt>& P0, const ts_signal& sig, double range,
               std::vector<int>* phi) {
    phi->assign(P0.size(), -1);
    const double thr = double(sig.threshold_rel) * range;
    for (size_t i = 0; i < P0.size(); ++i) {
      const Pt& p = P0[i];
      bool keep;
      if (p.ess) {
        keep = true;
      } else if (sig.mode == 1) {
        keep = false;
        for (int64_t q = 0; q < sig.n_signal && !keep; ++q)
          keep = sig.signal[q].dim == p.dim && sig.signal[q].birth_cell == p.bcell &&
                 sig.signal[q].death_cell == p.dcell;
      } else {
        const double pers = double(p.d) - double(p.b);
        const bool masked = (sig.nonsignal_dim_mask >> p.dim) & 1u;
        const bool below = pers < thr || (pers == thr && !sig.ties_signal);
        keep = !(masked && below);
      }
      if (keep) {
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

  void assign(const std::vector<Pt>& P, const std::vector<Pt>& Pp, const std::vector<int>& phip,
              std::vector<int>* phi, int64_t* n_still, int64_t* n_red) {
    phi->assign(P.size(), -1);
    // previous points grouped by key, in diagram order
    std::unordered_map<uint64_t, std::pair<int, int>> head;  // key -> (first, count)
    std::vector<int> chain(Pp.size(), -1), tail;
    std::unordered_map<uint64_t, int> last;
    head.reserve(Pp.size() * 2);
    for (size_t j = 0; j < Pp.size(); ++j) {
      const uint64_t k = pkey(Pp[j].dim, Pp[j].vb, Pp[j].vd);
      auto it = last.find(k);
      if (it == last.end()) {
        head[k] = {int(j), 1};
        last[k] = int(j);
      } else {
        chain[it->second] = int(j);
        it->second = int(j);
      }
    }
    std::vector<char> still(P.size(), 0), held(T.size(), 0);
    *n_still = 0;
    for (size_t i = 0; i < P.size(); ++i) {
      auto it = head.find(pkey(P[i].dim, P[i].vb, P[i].vd));
      if (it == head.end() || it->second.first < 0) continue;
      const int j = it->second.first;
      it->second.first = chain[j];
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
    for (int dim = 0; dim < 3; ++dim) {
      std::vector<int> pi, tj;
      std::vector<double> pb, pd, qb, qd;
      for (int i : red)
        if (P[i].dim == dim) {
          pi.push_back(i);
          pb.push_back(P[i].b);
          pd.push_back(P[i].d);
        }
      for (size_t j = 0; j < T.size(); ++j)
        if (!held[j] && !T[j].ess && T[j].dim == dim) {
          tj.push_back(int(j));
          qb.push_back(T[j].b);
          qd.push_back(T[j].d);
        }
      if (pi.empty()) continue;
      std::vector<int> m;
      assign_exact(pb, pd, qb, qd, &m);
      for (size_t s = 0; s < pi.size(); ++s) (*phi)[pi[s]] = m[s] >= 0 ? tj[m[s]] : -1;
    }
    canonical_form(P, red, T, phi);
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

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------- assignment

double assign_exact(const std::vector<double>& pb, const std::vector<double>& pd,
                    const std::vector<double>& qb, const std::vector<double>& qd,
                    std::vector<int>* match) {
  // Augmented bipartite graph: left = points (m) + diagonal copies of targets
  // (k); right = targets (k) + diagonal copies of points (m).  Edges:
  //   point i - target j        c(p_i, q_j), only if c < diag(p_i) + diag(q_j)
  //   point i - diag copy of i  diag(p_i)
  //   diag copy of j - target j diag(q_j)
  //   diag copy of j - diag copy of i   0, for the same (i, j) as above
  // (the last block only needs the pairs kept in the first one: a matching
  // that uses point i - target j can always pair the two diagonal copies).
  const int m = int(pb.size()), k = int(qb.size());
  match->assign(m, -1);
  const int N = m + k;
  if (N == 0) return 0.0;
  struct E {
    int to;
    double c;
  };
  std::vector<std::vector<E>> adj(N);
  std::vector<double> dp(m), dq(k);
  for (int i = 0; i < m; ++i) dp[i] = diag_cost(pb[i], pd[i]);
  for (int j = 0; j < k; ++j) dq[j] = diag_cost(qb[j], qd[j]);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < k; ++j) {
      const double c = pair_cost(pb[i], pd[i], qb[j], qd[j]);
      if (c < dp[i] + dq[j]) {
        adj[i].push_back({j, c});
        adj[m + j].push_back({k + i, 0.0});
      }
    }
    adj[i].push_back({k + i, dp[i]});
  }
  for (int j = 0; j < k; ++j) adj[m + j].push_back({j, dq[j]});

  // successive shortest augmenting paths with potentials (Dijkstra)
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<int> ml(N, -1), mr(N, -1);
  std::vector<double> mc(N, 0.0), hl(N, 0.0), hr(N, 0.0), dl(N), dr(N);
  std::vector<int> prev_r(N);
  std::vector<int> touched_l, touched_r;
  typedef std::pair<double, int> QI;  // (dist, node): node < N left, >= N right
  for (int s = 0; s < N; ++s) {
    std::fill(dl.begin(), dl.end(), INF);
    std::fill(dr.begin(), dr.end(), INF);
    std::priority_queue<QI, std::vector<QI>, std::greater<QI>> pq;
    dl[s] = 0.0;
    pq.push({0.0, s});
    int found = -1;
    while (!pq.empty()) {
      const QI top = pq.top();
      pq.pop();
      const double d = top.first;
      if (top.second < N) {
        const int l = top.second;
        if (d > dl[l]) continue;
        for (const E& e : adj[l]) {
          if (ml[l] == e.to) continue;
          const double nd = d + e.c + hl[l] - hr[e.to];
          if (nd < dr[e.to]) {
            dr[e.to] = nd;
            prev_r[e.to] = l;
            pq.push({nd, N + e.to});
          }
        }
      } else {
        const int r = top.second - N;
        if (d > dr[r]) continue;
        if (mr[r] < 0) {
          found = r;
          break;
        }
        const int l = mr[r];
        const double nd = d - mc[l] + hr[r] - hl[l];
        if (nd < dl[l]) {
          dl[l] = nd;
          pq.push({nd, l});
        }
      }
    }
    if (found < 0) throw Error(TS_ERR_INTERNAL, "assignment: no augmenting path");
    const double D = dr[found];
    for (int l = 0; l < N; ++l) hl[l] += std::min(dl[l], D);
    for (int r = 0; r < N; ++r) hr[r] += std::min(dr[r], D);
    // augment
    int r = found;
    while (true) {
      const int l = prev_r[r];
      const int old = ml[l];
      double c = 0;
      for (const E& e : adj[l])
        if (e.to == r) {
          c = e.c;
          break;
        }
      ml[l] = r;
      mr[r] = l;
      mc[l] = c;
      if (l == s) break;
      r = old;
    }
  }
  double total = 0;  // every left node is matched
  for (int l = 0; l < N; ++l) total += mc[l];
  for (int i = 0; i < m; ++i) (*match)[i] = ml[i] < k ? ml[i] : -1;
  return total;
}

// ---------------------------------------------------------------- loop

int simplify(ts_ctx* ctx, const float* f, const Grid& G, const ts_signal& sig,
             const ts_options& opt, float* g_out, ts_report* rep) {
  const double t0 = now_s();
  hipStream_t s = ctx->stream;
  const int n = G.n;
  std::memset(rep, 0, sizeof(*rep));
  float* x = dev<float>(ctx, "sim.x", n);
  float* f0 = dev<float>(ctx, "sim.f0", n);
  if (opt.inputs_on_device) {
    TS_HIP(hipMemcpyAsync(f0, f, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
  } else {
    TS_HIP(hipMemcpyAsync(f0, f, size_t(n) * 4, hipMemcpyHostToDevice, s));
  }
  TS_HIP(hipMemcpyAsync(x, f0, size_t(n) * 4, hipMemcpyDeviceToDevice, s));

  PersistenceResult R;
  double tp = now_s();
  compute_persistence(ctx, x, G, &R);  // also rejects non-finite values
  rep->persistence_s += now_s() - tp;

  // range of f0
  double range;
  {
    const int nb = 256;
    float* mm = dev<float>(ctx, "sim.mm", 2 * nb);
    k_minmax<<<nb, 256, 0, s>>>(f0, n, mm);
    std::vector<float> h(2 * nb);
    TS_HIP(hipMemcpyAsync(h.data(), mm, h.size() * 4, hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    double mn = h[0], mx = h[1];
    for (int b = 0; b < nb; ++b) {
      mn = std::min(mn, double(h[2 * b]));
      mx = std::max(mx, double(h[2 * b + 1]));
    }
    range = mx - mn;
  }
  const double tol = double(opt.cancel_tol_rel) * range;

  std::vector<Pt> P;
  fetch_points(ctx, R, x, &P);
  Solver S;
  std::vector<int> phi;
  S.targets(P, sig, range, &phi);
  const double L0 = S.loss(P, phi);
  double L = L0;
  auto done = [&](double Lc) {
    if (opt.stop_mode == 1) return Lc <= double(opt.loss_ratio_s) * L0;
    return S.max_diag_pers(P, phi) < tol;
  };
  int j = 0;
  int64_t n_still = int64_t(P.size()), n_red = 0;
  bool cancelled = opt.stop_mode == 0 && done(L);
  while (!cancelled && j < opt.j_max) {
    ++j;
    // ---- gradient step ----
    const double tu = now_s();
    {
      const int64_t np = int64_t(P.size());
      std::vector<int32_t> hvb(np), hvd(np);
      std::vector<float> htb(np), htd(np);
      for (int64_t i = 0; i < np; ++i) {
        hvb[i] = P[i].vb;
        hvd[i] = P[i].vd;
        if (phi[i] >= 0) {
          htb[i] = S.T[phi[i]].b;
          htd[i] = S.T[phi[i]].d;
        } else {
          const float mid = (P[i].b + P[i].d) * 0.5f;
          htb[i] = htd[i] = mid;
        }
      }
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
      k_step_keys<<<nblk(np), 256, 0, s>>>(dvb, dvd, np, keys, vals);
      const int vbits = 33 + 32 - __builtin_clz(uint32_t(std::max(n - 1, 1)));
      radix_sort_u64(ctx->ws, keys, vals, size_t(2 * np), 0, vbits, s);
      k_step_apply<<<nblk(2 * np), 256, 0, s>>>(keys, 2 * np, dtb, dtd, x, opt.alpha_b,
                                                opt.alpha_d);
      ctx->timer.stop();
      TS_HIP(hipGetLastError());
      TS_HIP(hipStreamSynchronize(s));
    }
    rep->update_s += now_s() - tu;
    // ---- persistence ----
    tp = now_s();
    compute_persistence(ctx, x, G, &R);
    std::vector<Pt> Pn;
    fetch_points(ctx, R, x, &Pn);
    rep->persistence_s += now_s() - tp;
    // ---- assignment ----
    const double ta = now_s();
    std::vector<int> phin;
    S.assign(Pn, P, phi, &phin, &n_still, &n_red);
    P.swap(Pn);
    phi.swap(phin);
    L = S.loss(P, phi);
    rep->assign_s += now_s() - ta;
    cancelled = done(L);
  }

  // ---- outputs and report ----
  std::vector<float> hx(n), hf(n);
  TS_HIP(hipMemcpyAsync(hx.data(), x, size_t(n) * 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipMemcpyAsync(hf.data(), f0, size_t(n) * 4, hipMemcpyDeviceToHost, s));
  if (opt.inputs_on_device)
    TS_HIP(hipMemcpyAsync(g_out, x, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
  TS_HIP(hipStreamSynchronize(s));
  if (!opt.inputs_on_device) std::memcpy(g_out, hx.data(), size_t(n) * 4);
  rep->iterations = j;
  rep->cancelled = cancelled ? 1 : 0;
  rep->loss0 = L0;
  rep->loss = L;
  {
    std::vector<char> used(S.T.size(), 0);
    for (int t : phi)
      if (t >= 0) used[t] = 1;
    double un = 0;
    for (size_t t = 0; t < S.T.size(); ++t)
      if (!used[t]) un += diag_cost(S.T[t].b, S.T[t].d);
    rep->energy = L + un;
  }
  double linf = 0, l2 = 0;
  for (int i = 0; i < n; ++i) {
    const double d = double(hx[i]) - double(hf[i]);
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
  for (const Pt& p : P)
    if (!p.ess) rep->n_pairs[p.dim]++;
  rep->n_still = n_still;
  rep->n_reduced = n_red;
  rep->n_targets = int64_t(S.T.size());
  rep->total_s = now_s() - t0;
  return cancelled ? TS_OK : TS_WARN_NOT_CANCELLED;
}

}  // namespace ts
