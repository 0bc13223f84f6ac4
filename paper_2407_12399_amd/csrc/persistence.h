// persistence.h -- device-resident persistence map of a field on the
// Freudenthal triangulation (host-side interface of persistence.hip).
#pragma once

#include <vector>

#include "internal.h"

namespace ts {

// Fields stored one after another in one device buffer: field i has grid
// grids[i] and holds vertices [base[i], base[i + 1]) (base has nf + 1 entries).
struct Batch {
  std::vector<Grid> grids;
  std::vector<int64_t> base;
};

// Everything the persistence map leaves on the device.  Pointers live in the
// context workspace and stay valid until the next call that reuses it.
struct PersistenceResult {
  Grid g{};
  // vertex order (Sec. 2.2)
  int32_t* order = nullptr;  // [n]
  int32_t* rank = nullptr;   // [n]
  // lower-star gradient (Sec. 4.2): per-vertex pairing code and the vertex
  // reached by the descending gradient step (itself for a minimum)
  uint4* code = nullptr;     // [n]
  int32_t* down = nullptr;   // [n]
  // critical cells per dim, sorted by lexicographic key
  int64_t ncrit[4] = {0, 0, 0, 0};
  uint64_t* ckey[4] = {};    // key = rank(highest vertex) << 12 | local key
  int32_t* cid[4] = {};      // canonical ids
  // persistence pairs of critical cells (+ the essential class, last)
  int64_t npairs = 0;
  int32_t* pdim = nullptr;
  int32_t* pbirth = nullptr;  // canonical id
  int32_t* pdeath = nullptr;  // canonical id, -1 for the essential class
  uint64_t* pbkey = nullptr;  // lexicographic key of the birth cell
  uint64_t* pdkey = nullptr;  // of the death cell (n-1 << 12 for the essential)
  // diagram: pair indices in diagram order, v_birth != v_death or essential
  int64_t ndiag = 0;
  uint32_t* diag = nullptr;
  // round counts of the iterative stages (diagnostics)
  int rounds_d0 = 0, rounds_d2 = 0, rounds_d1 = 0;
  // vertices whose lower star was processed by the last call (n unless the
  // fast update ran)
  int64_t n_regrad = 0;
  // set when the call finished; the fast update needs a complete previous map
  bool complete = false;
  // field dims (3 per field) of the last call, and the number of fields
  std::vector<int64_t> layout;
  int nfields = 1;
};

// Vertex order only (K1 + K2).
void compute_order(ts_ctx* ctx, const float* f, int n, int32_t* order, int32_t* rank);
// The vertex order with no device allocation: temporaries in a static device
// array (at most 2^21 vertices); f, order, rank are device pointers.
void order_noalloc(const float* f, int64_t n, int32_t* order, int32_t* rank, hipStream_t s);

// The whole persistence map (K1..K8) of a device field.  With `changed`
// (device, n bytes, nonzero where the value differs from the field of the
// previous call on the same R and context), the gradient is updated instead of
// recomputed (Sec. 4.2): only vertices with a changed value in their closed
// star run the lower-star loop; the result is the same as a full map.  Nothing
// else may use the context's workspace between the two calls.
// With `batch`, f holds several fields one after another (g.n = their total,
// g's dims unused) and the result is that of every field's own map, in the
// batch's vertex and cell id spaces (ids offset by the field's base).
void compute_persistence(ts_ctx* ctx, const float* f, const Grid& g, PersistenceResult* R,
                         const uint8_t* changed = nullptr, const Batch* batch = nullptr);

// ts_pair records of the diagram (diagram order) or of all pairs (device).
void pair_records(ts_ctx* ctx, const PersistenceResult& R, const float* f, bool diagram_only,
                  ts_pair* out_dev);

// The diagram of a batch split by field on the device: out_dev holds field
// 0's records, then field 1's, ..., each in its field's diagram order and with
// field-local ids; counts (host, nf entries) receives the sizes.
void batch_diagram_records(ts_ctx* ctx, const PersistenceResult& R, const float* f,
                           const Batch& B, ts_pair* out_dev, int64_t* counts);

// Dense gradient partner arrays (device outputs of sizes n, 7n, 12n).
void decode_gradient(ts_ctx* ctx, const PersistenceResult& R, int32_t* vup, int32_t* eup,
                     int32_t* tup);

}  // namespace ts
