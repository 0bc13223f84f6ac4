// api.cpp -- C ABI of the topsimp library (context, workspace, stage calls).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "persistence.h"
#include "solver.h"
#include "unet.h"

namespace ts {

void* Workspace::get(const std::string& name, size_t bytes) {
  Buf& b = bufs[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) {
    // previous users on the stream must be done before the memory is reused
    TS_HIP(hipDeviceSynchronize());
    TS_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  want = (want + 255) & ~size_t(255);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    throw Error(TS_ERR_OOM, "hipMalloc(" + std::to_string(want) + ") for " + name + ": " +
                                hipGetErrorString(e));
  }
  b.bytes = want;
  return b.p;
}

void* Workspace::host(const std::string& name, size_t bytes) {
  Buf& b = host_bufs[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) {
    TS_HIP(hipDeviceSynchronize());
    TS_HIP(hipHostFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 4096);
  want += want / 8;  // room to grow a little without a new allocation
  hipError_t e = hipHostMalloc(&b.p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    b.p = nullptr;
    throw Error(TS_ERR_OOM, "hipHostMalloc(" + std::to_string(want) + ") for " + name + ": " +
                                hipGetErrorString(e));
  }
  b.bytes = want;
  return b.p;
}

void Workspace::release() {
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs.clear();
  for (auto& kv : host_bufs)
    if (kv.second.p) (void)hipHostFree(kv.second.p);
  host_bufs.clear();
}

size_t Workspace::total_bytes() const {
  size_t s = 0;
  for (const auto& kv : bufs) s += kv.second.bytes;
  return s;
}

void Timer::reset() {
  for (auto& e : begin) (void)hipEventDestroy(e);
  for (auto& e : end) (void)hipEventDestroy(e);
  begin.clear();
  end.clear();
  names.clear();
  open.clear();
}

void Timer::start(const std::string& name) {
  if (!enabled) return;
  hipEvent_t a, b;
  TS_HIP(hipEventCreate(&a));
  TS_HIP(hipEventCreate(&b));
  TS_HIP(hipEventRecord(a, stream));
  begin.push_back(a);
  end.push_back(b);
  names.push_back(name);
  open.push_back(name);
}

void Timer::stop() {
  if (!enabled || open.empty()) return;
  TS_HIP(hipEventRecord(end.back(), stream));
  open.pop_back();
}

void Timer::collect(std::vector<std::string>* names_out, std::vector<double>* ms_out) {
  names_out->clear();
  ms_out->clear();
  if (begin.empty()) return;
  TS_HIP(hipStreamSynchronize(stream));
  for (size_t i = 0; i < begin.size(); ++i) {
    float ms = 0.f;
    TS_HIP(hipEventElapsedTime(&ms, begin[i], end[i]));
    auto it = std::find(names_out->begin(), names_out->end(), names[i]);
    if (it == names_out->end()) {
      names_out->push_back(names[i]);
      ms_out->push_back(ms);
    } else {
      (*ms_out)[it - names_out->begin()] += ms;
    }
  }
}

void Timer::destroy() { reset(); }

Grid make_grid(const int64_t dims[3]) {
  if (!dims) throw Error(TS_ERR_ARG, "dims is NULL");
  for (int i = 0; i < 3; ++i)
    if (dims[i] < 2) throw Error(TS_ERR_ARG, "every dimension must be >= 2");
  const int64_t n = dims[0] * dims[1] * dims[2];
  if (dims[0] > (1 << 25) || dims[1] > (1 << 25) || dims[2] > (1 << 25) || n > (int64_t(1) << 25))
    throw Error(TS_ERR_ARG, "grid larger than 2^25 vertices");
  Grid g;
  g.Lx = int(dims[0]);
  g.Ly = int(dims[1]);
  g.Lz = int(dims[2]);
  g.n = int(n);
  return g;
}

// Device copy of the field (or the caller's device pointer).
const float* device_field(ts_ctx* ctx, const float* f, int64_t n, int on_device) {
  if (!f) throw Error(TS_ERR_ARG, "field pointer is NULL");
  if (on_device) return f;
  float* d = ctx->ws.get<float>("api.field", n);
  TS_HIP(hipMemcpyAsync(d, f, n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  return d;
}

void finish_timing(ts_ctx* ctx) {
  ctx->timer.collect(&ctx->stage_names_store, &ctx->stage_ms);
  ctx->stage_names.clear();
  for (const auto& s : ctx->stage_names_store) ctx->stage_names.push_back(s.c_str());
  ctx->stage_names.push_back(nullptr);
}

// Host records of the pairs (all, or the diagram subset in diagram order),
// assembled on the device.
// The records are copied straight into the caller's array (at full link
// speed when it is pinned memory); returns the count, and copies nothing when
// it exceeds the capacity.
int64_t pairs_to_host(ts_ctx* ctx, const PersistenceResult& R, const float* f_dev,
                      bool diagram_only, ts_pair* dst, int64_t capacity) {
  hipStream_t s = ctx->stream;
  const int64_t n = diagram_only ? R.ndiag : R.npairs;
  if (n > capacity) return n;
  if (n > 0 && !dst) throw Error(TS_ERR_ARG, "out is NULL");
  ts_pair* d = ctx->ws.get<ts_pair>("api.records", n + 1);
  pair_records(ctx, R, f_dev, diagram_only, d);
  if (n) TS_HIP(hipMemcpyAsync(dst, d, n * sizeof(ts_pair), hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  if (!diagram_only)
    std::sort(dst, dst + n, [](const ts_pair& a, const ts_pair& b) {
      if (a.dim != b.dim) return a.dim < b.dim;
      if (a.birth_cell != b.birth_cell) return a.birth_cell < b.birth_cell;
      return a.death_cell < b.death_cell;
    });
  return n;
}

void pairs_to_host(ts_ctx* ctx, const PersistenceResult& R, const float* f_dev, bool diagram_only,
                   std::vector<ts_pair>* out) {
  const int64_t n = diagram_only ? R.ndiag : R.npairs;
  out->resize(n);
  pairs_to_host(ctx, R, f_dev, diagram_only, out->data(), n);
}

// Layout of a batch of fields stored one after another.
Batch make_batch(int32_t nf, const int64_t* dims) {
  if (nf < 1 || !dims) throw Error(TS_ERR_ARG, "a batch needs at least one field");
  Batch B;
  B.base.push_back(0);
  for (int32_t i = 0; i < nf; ++i) {
    B.grids.push_back(make_grid(dims + 3 * i));
    B.base.push_back(B.base.back() + B.grids.back().n);
    if (B.base.back() > (int64_t(1) << 25))
      throw Error(TS_ERR_ARG, "batch larger than 2^25 vertices");
  }
  return B;
}

// The fields of a batch copied one after another into one device buffer.
float* batch_field(ts_ctx* ctx, const Batch& B, const float* const* f, int on_device,
                   const char* name) {
  if (!f) throw Error(TS_ERR_ARG, "field list is NULL");
  const int nf = int(B.grids.size());
  float* d = ctx->ws.get<float>(name, B.base[nf]);
  for (int i = 0; i < nf; ++i) {
    if (!f[i]) throw Error(TS_ERR_ARG, "field pointer is NULL");
    TS_HIP(hipMemcpyAsync(d + B.base[i], f[i], size_t(B.grids[i].n) * sizeof(float),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          ctx->stream));
  }
  return d;
}

// Whether [a, a + na) and [b, b + nb) (float counts) share memory.
bool overlaps(const float* a, int64_t na, const float* b, int64_t nb) {
  const uintptr_t a0 = uintptr_t(a), a1 = a0 + uintptr_t(na) * sizeof(float);
  const uintptr_t b0 = uintptr_t(b), b1 = b0 + uintptr_t(nb) * sizeof(float);
  return a0 < b1 && b0 < a1;
}

void check_solver_args(const ts_signal* sig, const ts_options* opt) {
  if (!sig || !opt) throw Error(TS_ERR_ARG, "null argument");
  if (!(opt->assign_precision >= 0) || !std::isfinite(opt->assign_precision))
    throw Error(TS_ERR_ARG, "assign_precision must be finite and >= 0");
  if (opt->j_max < 0 || opt->stop_mode < 0 || opt->stop_mode > 1)
    throw Error(TS_ERR_ARG, "bad options");
  if (opt->trace && opt->trace_cap < 0) throw Error(TS_ERR_ARG, "bad trace capacity");
  if (sig->mode != 0 && sig->mode != 1) throw Error(TS_ERR_ARG, "bad signal mode");
  if (sig->mode == 1 && sig->n_signal > 0 && !sig->signal)
    throw Error(TS_ERR_ARG, "signal list is NULL");
}

template <class F>
int guarded(ts_ctx* ctx, F&& fn) {
  if (!ctx) return TS_ERR_ARG;
  try {
    TS_HIP(hipSetDevice(ctx->device));
    ctx->err.clear();
    return fn();
  } catch (const Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return TS_ERR_OOM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return TS_ERR_INTERNAL;
  }
}

}  // namespace ts

using namespace ts;

extern "C" {

int ts_create(ts_ctx** out, int device, void* hip_stream) {
  if (!out) return TS_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return TS_ERR_HIP;
  if (device < 0 || device >= count) return TS_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return TS_ERR_HIP;
  ts_ctx* c = new (std::nothrow) ts_ctx;
  if (!c) return TS_ERR_OOM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->timer.stream = c->stream;
  *out = c;
  return TS_OK;
}

int ts_destroy(ts_ctx* ctx) {
  if (!ctx) return TS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->timer.destroy();
  ctx->ws.release();
  delete ctx;
  return TS_OK;
}

const char* ts_last_error(const ts_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int ts_order(ts_ctx* ctx, const float* f, int64_t n, int32_t on_device, int32_t* order,
             int32_t* rank) {
  return guarded(ctx, [&]() {
    if (!order || !rank || n < 1 || n > (int64_t(1) << 25))
      throw Error(TS_ERR_ARG, "bad arguments");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, n, on_device);
    int32_t* od = on_device ? order : ctx->ws.get<int32_t>("api.order", n);
    int32_t* rd = on_device ? rank : ctx->ws.get<int32_t>("api.rank", n);
    compute_order(ctx, fd, int(n), od, rd);
    if (!on_device) {
      TS_HIP(hipMemcpyAsync(order, od, n * 4, hipMemcpyDeviceToHost, ctx->stream));
      TS_HIP(hipMemcpyAsync(rank, rd, n * 4, hipMemcpyDeviceToHost, ctx->stream));
    }
    TS_HIP(hipStreamSynchronize(ctx->stream));
    finish_timing(ctx);
    return TS_OK;
  });
}

int ts_gradient(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
                int32_t* vup, int32_t* eup, int32_t* tup) {
  return guarded(ctx, [&]() {
    const Grid g = make_grid(dims);
    if (!vup || !eup || !tup) throw Error(TS_ERR_ARG, "null output");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, g.n, on_device);
    PersistenceResult R;
    compute_persistence(ctx, fd, g, &R);
    int32_t* v = ctx->ws.get<int32_t>("api.vup", g.n);
    int32_t* e = ctx->ws.get<int32_t>("api.eup", 7 * int64_t(g.n));
    int32_t* t = ctx->ws.get<int32_t>("api.tup", 12 * int64_t(g.n));
    decode_gradient(ctx, R, v, e, t);
    TS_HIP(hipMemcpyAsync(vup, v, size_t(g.n) * 4, hipMemcpyDeviceToHost, ctx->stream));
    TS_HIP(hipMemcpyAsync(eup, e, size_t(g.n) * 28, hipMemcpyDeviceToHost, ctx->stream));
    TS_HIP(hipMemcpyAsync(tup, t, size_t(g.n) * 48, hipMemcpyDeviceToHost, ctx->stream));
    TS_HIP(hipStreamSynchronize(ctx->stream));
    finish_timing(ctx);
    return TS_OK;
  });
}

int ts_critical(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
                int32_t* out_dim, int64_t* out_id, int64_t capacity, int64_t counts[4]) {
  return guarded(ctx, [&]() {
    const Grid g = make_grid(dims);
    if (!counts) throw Error(TS_ERR_ARG, "counts is NULL");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, g.n, on_device);
    PersistenceResult R;
    compute_persistence(ctx, fd, g, &R);
    int64_t total = 0;
    for (int d = 0; d < 4; ++d) {
      counts[d] = R.ncrit[d];
      total += R.ncrit[d];
    }
    finish_timing(ctx);
    if (total > capacity) {
      ctx->err = "capacity too small";
      return int(TS_ERR_CAPACITY);
    }
    if (!out_dim || !out_id) throw Error(TS_ERR_ARG, "null output");
    int64_t k = 0;
    for (int d = 0; d < 4; ++d) {
      std::vector<int32_t> ids(R.ncrit[d]);
      if (R.ncrit[d])
        TS_HIP(hipMemcpy(ids.data(), R.cid[d], R.ncrit[d] * 4, hipMemcpyDeviceToHost));
      for (int32_t id : ids) {
        out_dim[k] = d;
        out_id[k++] = id;
      }
    }
    return int(TS_OK);
  });
}

int ts_pairs(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
             ts_pair* out, int64_t capacity, int64_t* n_out) {
  return guarded(ctx, [&]() {
    const Grid g = make_grid(dims);
    if (!n_out) throw Error(TS_ERR_ARG, "n_out is NULL");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, g.n, on_device);
    PersistenceResult R;
    compute_persistence(ctx, fd, g, &R);
    const int64_t n = pairs_to_host(ctx, R, fd, false, out, capacity);
    finish_timing(ctx);
    *n_out = n;
    if (n > capacity) {
      ctx->err = "capacity too small";
      return int(TS_ERR_CAPACITY);
    }
    return int(TS_OK);
  });
}

int ts_diagram(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
               ts_pair* out, int64_t capacity, int64_t* n_out) {
  return guarded(ctx, [&]() {
    const Grid g = make_grid(dims);
    if (!n_out) throw Error(TS_ERR_ARG, "n_out is NULL");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, g.n, on_device);
    PersistenceResult R;
    compute_persistence(ctx, fd, g, &R);
    const int64_t n = pairs_to_host(ctx, R, fd, true, out, capacity);
    finish_timing(ctx);
    *n_out = n;
    if (n > capacity) {
      ctx->err = "capacity too small";
      return int(TS_ERR_CAPACITY);
    }
    return int(TS_OK);
  });
}

int ts_diagram_batch(ts_ctx* ctx, int32_t nf, const float* const* f, const int64_t* dims,
                     int32_t on_device, ts_pair* out, int64_t capacity, int64_t* counts) {
  return guarded(ctx, [&]() {
    const Batch B = make_batch(nf, dims);
    if (!counts) throw Error(TS_ERR_ARG, "counts is NULL");
    ctx->timer.reset();
    const float* fd = batch_field(ctx, B, f, on_device, "api.batch_field");
    Grid g{0, 0, 0, int(B.base[nf])};
    PersistenceResult R;
    compute_persistence(ctx, fd, g, &R, nullptr, &B);
    // split by field on the device (diagram order restricted to a field is
    // that field's own diagram order), then one copy into the caller's array
    const int64_t total = R.ndiag;
    ts_pair* d = ctx->ws.get<ts_pair>("api.batch_records", size_t(total) + 1);
    batch_diagram_records(ctx, R, fd, B, d, counts);
    finish_timing(ctx);
    if (total > capacity) {
      ctx->err = "capacity too small";
      return int(TS_ERR_CAPACITY);
    }
    if (!out && total > 0) throw Error(TS_ERR_ARG, "out is NULL");
    if (total > 0)
      TS_HIP(hipMemcpyAsync(out, d, size_t(total) * sizeof(ts_pair), hipMemcpyDeviceToHost,
                            ctx->stream));
    TS_HIP(hipStreamSynchronize(ctx->stream));
    return int(TS_OK);
  });
}

int ts_unet_param_count(int64_t* n) {
  if (!n) return TS_ERR_ARG;
  *n = unet_param_count();
  return TS_OK;
}

namespace {
void unet_dims(const int64_t dims[3], int* D, int* H, int* W) {
  if (!dims) throw Error(TS_ERR_ARG, "dims is NULL");
  for (int i = 0; i < 3; ++i)
    if (dims[i] < 4 || dims[i] % 4 != 0 || dims[i] > 4096)
      throw Error(TS_ERR_ARG, "network sizes must be multiples of 4 in [4, 4096]");
  if (dims[0] * dims[1] * dims[2] > (int64_t(1) << 25))
    throw Error(TS_ERR_ARG, "volume larger than 2^25 voxels");
  *W = int(dims[0]);
  *H = int(dims[1]);
  *D = int(dims[2]);
}
}  // namespace

int ts_unet_forward(ts_ctx* ctx, const float* params, const float* input, const int64_t dims[3],
                    float* out) {
  return guarded(ctx, [&]() {
    int D, H, W;
    unet_dims(dims, &D, &H, &W);
    if (!params || !input || !out) throw Error(TS_ERR_ARG, "null argument");
    unet_forward(ctx, params, input, D, H, W, out);
    TS_HIP(hipStreamSynchronize(ctx->stream));
    return int(TS_OK);
  });
}

int ts_unet_backward(ts_ctx* ctx, const float* params, const float* input, const float* target,
                     const int64_t dims[3], float* grad, double* loss) {
  return guarded(ctx, [&]() {
    int D, H, W;
    unet_dims(dims, &D, &H, &W);
    if (!params || !input || !target || !grad || !loss) throw Error(TS_ERR_ARG, "null argument");
    *loss = unet_backward(ctx, params, input, target, D, H, W, grad);
    return int(TS_OK);
  });
}

int ts_unet_adam(ts_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t n,
                 int64_t step, float lr, float beta1, float beta2, float eps) {
  return guarded(ctx, [&]() {
    if (!params || !grad || !m || !v || n < 0 || step < 1) throw Error(TS_ERR_ARG, "bad arguments");
    unet_adam(ctx, params, grad, m, v, n, step, lr, beta1, beta2, eps);
    return int(TS_OK);
  });
}

int ts_simplify_batch(ts_ctx* ctx, int32_t nf, const float* const* f, const int64_t* dims,
                      const ts_signal* sig, const ts_options* opt, float* const* g,
                      ts_report* reps) {
  return guarded(ctx, [&]() {
    const Batch B = make_batch(nf, dims);
    check_solver_args(sig, opt);
    if (sig->mode != 0) throw Error(TS_ERR_ARG, "a batch takes the threshold signal mode only");
    if (opt->init) throw Error(TS_ERR_ARG, "a batch takes no start field");
    if (opt->trace) throw Error(TS_ERR_ARG, "a batch takes no trace");
    if (!f || !g || !reps) throw Error(TS_ERR_ARG, "null argument");
    for (int i = 0; i < nf; ++i)
      if (!f[i] || !g[i]) throw Error(TS_ERR_ARG, "null field pointer");
    for (int i = 0; i < nf; ++i)
      for (int k = 0; k < nf; ++k) {
        if (overlaps(g[i], B.grids[i].n, f[k], B.grids[k].n))
          throw Error(TS_ERR_ARG, "an output must not overlap an input");
        if (k != i && overlaps(g[i], B.grids[i].n, g[k], B.grids[k].n))
          throw Error(TS_ERR_ARG, "outputs must not overlap");
      }
    ctx->timer.reset();
    const int rc = simplify_batch(ctx, B, f, *sig, *opt, g, reps);
    finish_timing(ctx);
    return rc;
  });
}

int ts_simplify(ts_ctx* ctx, const float* f, const int64_t dims[3], const ts_signal* sig,
                const ts_options* opt, float* g, ts_report* rep) {
  return guarded(ctx, [&]() {
    const Grid grid = make_grid(dims);
    check_solver_args(sig, opt);
    if (!g || !rep || !f) throw Error(TS_ERR_ARG, "null argument");
    if (overlaps(f, grid.n, g, grid.n)) throw Error(TS_ERR_ARG, "g must not overlap f");
    if (opt->init && overlaps(opt->init, grid.n, g, grid.n))
      throw Error(TS_ERR_ARG, "g must not overlap the start field");
    ctx->timer.reset();
    const int rc = simplify(ctx, f, grid, *sig, *opt, g, rep);
    finish_timing(ctx);
    return rc;
  });
}

int ts_signal_mask(ts_ctx* ctx, const float* f, const int64_t dims[3], const ts_signal* sig,
                   int32_t on_device, float* mask, int64_t* n_signal) {
  return guarded(ctx, [&]() {
    const Grid grid = make_grid(dims);
    if (!sig || !mask) throw Error(TS_ERR_ARG, "null argument");
    if (sig->mode != 0 && sig->mode != 1) throw Error(TS_ERR_ARG, "bad signal mode");
    if (sig->mode == 1 && sig->n_signal > 0 && !sig->signal)
      throw Error(TS_ERR_ARG, "signal list is NULL");
    if (!f || overlaps(mask, grid.n, f, grid.n))
      throw Error(TS_ERR_ARG, "mask must not overlap f");
    ctx->timer.reset();
    const float* fd = device_field(ctx, f, grid.n, on_device);
    const int64_t c = signal_mask(ctx, fd, grid, *sig, mask, on_device);
    finish_timing(ctx);
    if (n_signal) *n_signal = c;
    return int(TS_OK);
  });
}

int ts_assign(int64_t n_pts, const double* pb, const double* pd, int64_t n_tgt, const double* qb,
              const double* qd, int32_t* match, double* cost) {
  if (n_pts < 0 || n_tgt < 0 || !match || !cost) return TS_ERR_ARG;
  if ((n_pts > 0 && (!pb || !pd)) || (n_tgt > 0 && (!qb || !qd))) return TS_ERR_ARG;
  try {
    std::vector<double> PB(pb, pb + n_pts), PD(pd, pd + n_pts), QB(qb, qb + n_tgt),
        QD(qd, qd + n_tgt);
    std::vector<int> m;
    *cost = assign_reduced(PB, PD, QB, QD, &m);
    for (int64_t i = 0; i < n_pts; ++i) match[i] = m[i];
    return TS_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return TS_ERR_INTERNAL;
  }
}

int ts_assign_auction(int64_t n_pts, const double* pb, const double* pd, int64_t n_tgt,
                      const double* qb, const double* qd, double rel_precision, int32_t* match,
                      double* cost) {
  if (n_pts < 0 || n_tgt < 0 || !match || !cost) return TS_ERR_ARG;
  if ((n_pts > 0 && (!pb || !pd)) || (n_tgt > 0 && (!qb || !qd))) return TS_ERR_ARG;
  if (!(rel_precision >= 0) || !std::isfinite(rel_precision)) return TS_ERR_ARG;
  try {
    std::vector<double> PB(pb, pb + n_pts), PD(pd, pd + n_pts), QB(qb, qb + n_tgt),
        QD(qd, qd + n_tgt);
    std::vector<int> m;
    *cost = assign_reduced(PB, PD, QB, QD, &m, rel_precision, true);
    for (int64_t i = 0; i < n_pts; ++i) match[i] = m[i];
    return TS_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return TS_ERR_INTERNAL;
  }
}

int ts_order_noalloc(const float* f, int64_t n, int32_t* order, int32_t* rank,
                     void* hip_stream) {
  try {
    if (!f || !order || !rank || n < 1) return TS_ERR_ARG;
    const float* fo = reinterpret_cast<const float*>(order);
    const float* fr = reinterpret_cast<const float*>(rank);
    if (overlaps(f, n, fo, n) || overlaps(f, n, fr, n) || overlaps(fo, n, fr, n))
      return TS_ERR_ARG;
    order_noalloc(f, n, order, rank, static_cast<hipStream_t>(hip_stream));
    return TS_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return TS_ERR_INTERNAL;
  }
}

int ts_stage_times(const ts_ctx* ctx, const char* const** names, const double** ms) {
  if (!ctx || !names || !ms) return TS_ERR_ARG;
  *names = ctx->stage_names.empty() ? nullptr : ctx->stage_names.data();
  *ms = ctx->stage_ms.data();
  return int(ctx->stage_ms.size());
}

int ts_launch_choices(ts_ctx* ctx, const char* const** keys, const int** choices) {
  if (!ctx || !keys || !choices) return TS_ERR_ARG;
  ctx->tuner_keys_store.clear();
  ctx->tuner_choices.clear();
  for (const auto& kv : ctx->tuner.entries) {
    ctx->tuner_keys_store.push_back(kv.first);
    ctx->tuner_choices.push_back(kv.second.best);
  }
  ctx->tuner_keys.clear();
  for (const auto& k : ctx->tuner_keys_store) ctx->tuner_keys.push_back(k.c_str());
  ctx->tuner_keys.push_back(nullptr);
  *keys = ctx->tuner_keys.data();
  *choices = ctx->tuner_choices.data();
  return int(ctx->tuner_choices.size());
}

}  // extern "C"
