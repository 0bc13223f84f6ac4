/*
 * topsimp.h -- C ABI of the MI355X (gfx950) topological-simplification
 * library.
 *
 * Method: Kissi, Pont, Levine, Tierny, "A Practical Solver for Scalar Data
 * Topological Simplification" (arXiv 2407.12399).  The library computes the
 * persistence diagram of a PL scalar field on the Freudenthal triangulation
 * of a 3D regular grid (Sec. 2.1-2.2) with the discrete-gradient approach of
 * Sec. 4.2, and runs the simplification solver of Alg. 1 with the direct
 * gradient step of Sec. 4.1 and the still-pair assignment reuse of Sec. 4.3.
 * Every step of the persistence map, the still-pair join and the update runs
 * in the library's HIP kernels on one GPU; the reduced W2 assignment (Eq. 1
 * with q = 2 on the pairs that are not still) runs on the host.
 *
 * Conventions
 *  - Field: float32, layout [Lz][Ly][Lx] (x fastest), vertex id
 *    v = x + Lx*(y + Ly*z).  dims = {Lx, Ly, Lz}, each >= 2, Lx*Ly*Lz <= 2^25.
 *  - Triangulation: Freudenthal/Kuhn.  A cell anchored at vertex u is
 *    {u + c0, ..., u + ck} with 0 = c0 < c1 < ... < ck <= (1,1,1) a chain of
 *    unit-cube corners (corner mask bit0 = x, bit1 = y, bit2 = z).  Canonical
 *    ids: edge 7u+t, triangle 12u+t, tetrahedron 6u+t with types
 *      edge t:      c1 = t+1
 *      triangle t:  (c1,c2) in (1,3)(2,3)(1,5)(4,5)(2,6)(4,6)
 *                              (1,7)(2,7)(3,7)(4,7)(5,7)(6,7)
 *      tet t:       (c1,c2,7) with (c1,c2) in (1,3)(1,5)(2,3)(2,6)(4,5)(4,6)
 *  - Vertex order (Sec. 2.1-2.2): (value, id) ascending, -0.0 equal to +0.0.
 *  - Lexicographic filtration (Sec. 2.2): cells compare by the ranks of their
 *    vertices sorted decreasingly, a proper prefix first.
 *
 * Memory and streams
 *  - A context owns a HIP stream (the caller's, or the null stream) and a
 *    device workspace that grows on demand and is freed by ts_destroy.
 *  - Pointers marked "device or host" are read as device pointers when
 *    `inputs_on_device` (options) / `on_device` (arguments) is 1, otherwise as
 *    host pointers.  Device pointers must be valid on the context's device and
 *    are accessed in order on the context's stream.
 *  - Calls are synchronous: on return every output is written.
 *  - A context is not thread-safe; use one context per host thread.
 *
 * Status codes: every function returns one of the TS_* codes below; the
 * message of the last error is available from ts_last_error.
 */
#ifndef TOPSIMP_H
#define TOPSIMP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TS_OK = 0,
  TS_WARN_NOT_CANCELLED = 1, /* j_max reached before the stop rule held */
  TS_ERR_ARG = -1,           /* null pointer, bad dims, aliasing, bad option */
  TS_ERR_NONFINITE = -2,     /* NaN or Inf in the field */
  TS_ERR_OOM = -3,           /* device allocation failed */
  TS_ERR_HIP = -4,           /* HIP runtime error */
  TS_ERR_CAPACITY = -5,      /* output buffer too small (*n_out = required) */
  TS_ERR_INTERNAL = -6       /* an internal consistency check failed */
};

/* One persistence pair (Sec. 2.2), 48 bytes. */
typedef struct {
  int32_t dim;        /* 0 min-saddle, 1 saddle-saddle, 2 saddle-max */
  int32_t essential;  /* 1: the infinite class (dim 0); death_cell = -1,
                         v_death = last vertex of the order */
  int64_t birth_cell; /* canonical id of the birth simplex (dimension dim) */
  int64_t death_cell; /* canonical id of the death simplex (dimension dim+1) */
  int64_t v_birth;    /* highest vertex of the birth simplex */
  int64_t v_death;    /* highest vertex of the death simplex */
  float birth;        /* f(v_birth) */
  float death;        /* f(v_death) */
} ts_pair;

/* Signal selection (Sec. 3): which pairs of D(f0) are kept. */
typedef struct {
  int32_t mode;                /* 0: persistence threshold, 1: explicit list */
  float threshold_rel;         /* threshold = threshold_rel * (max f0 - min f0) */
  uint32_t nonsignal_dim_mask; /* bit k set: dim-k pairs below the threshold are
                                  non-signal; pairs of other dims are signal */
  int32_t ties_signal;         /* persistence == threshold: 1 signal, 0 non-signal */
  const ts_pair* signal;       /* mode 1: host array of signal pairs, matched on
                                  (dim, birth_cell, death_cell); others non-signal */
  int64_t n_signal;
} ts_signal;

/* Solver options (Sec. 4.1, Sec. 5). */
typedef struct {
  float alpha_b, alpha_d;  /* step sizes of the birth / death gradients (0.5, 0.5) */
  int32_t j_max;           /* iteration cap (1000) */
  int32_t stop_mode;       /* 0: every diagonal-assigned point has persistence
                                 < cancel_tol_rel * range (full cancellation)
                              1: loss <= loss_ratio_s * loss at iteration 0 */
  float cancel_tol_rel;    /* 1e-6 */
  float loss_ratio_s;      /* 0.01 */
  int32_t inputs_on_device; /* f and g are device pointers */
  float assign_precision;  /* 0: the reduced assignment is exact (the default; see
                              ts_assign).  > 0: an auction for
                              every size, stopped once its W2^2 total is within
                              (1 + assign_precision)^2 of a dual lower bound; the
                              paper runs 0.01 (Sec. 5).  Results then can differ
                              from the exact optimum. */
  int32_t full_gradient;   /* 0: after each update, the discrete gradient is recomputed only
                              for vertices with a changed value in their closed star
                              (the fast update of Sec. 4.2; same result).  1: the whole
                              gradient is recomputed every iteration. */
  const float* init;       /* NULL, or a start field g0 (n floats, same memory kind as f):
                              the solve starts from g0 (e.g. the warm-start network's
                              proposal) with the targets of D(f0), unless the loss of
                              g0 exceeds the loss of f0.  Single-field solves only. */
  double* trace;           /* NULL, or a host array of 4 * trace_cap doubles: entry j
                              (j = 0 .. iterations, up to trace_cap entries) holds the
                              wall seconds since the call began, the loss L_j, the
                              largest persistence among diagonal-assigned points and
                              the cumulative assignment seconds, after iteration j
                              (j = 0: the state of the start field).  Single-field
                              solves only. */
  int64_t trace_cap;
} ts_options;

typedef struct {
  int32_t iterations;       /* gradient steps performed */
  int32_t cancelled;        /* 1 if the stop rule held */
  double loss0, loss;       /* loss at iteration 0 / at the end */
  double energy;            /* loss + diagonal cost of unmatched targets */
  double linf, l2;          /* ||f-g||_inf, ||f-g||_2 */
  double max_nonsignal_pers; /* largest persistence among diagonal-assigned points */
  double max_signal_disp;   /* largest distance of a target-assigned point to its target */
  double range;             /* max(f0) - min(f0) */
  int64_t n_pairs[3];       /* final diagram size per dimension (finite pairs) */
  int64_t n_still;          /* still pairs at the last iteration */
  int64_t n_reduced;        /* points of the last reduced assignment problem */
  int64_t n_targets;        /* |D_T| */
  double total_s;           /* wall time of the call */
  double persistence_s;     /* time in the persistence map (all iterations) */
  double assign_s;          /* time in the still join + assignment */
  double update_s;          /* time in the gradient step */
  int64_t n_regradient;     /* vertices whose lower star was processed, summed over the
                               maps after the first (n per map with full_gradient) */
  int32_t init_used;        /* 1 if the solve started from options.init */
} ts_report;

typedef struct ts_ctx ts_ctx;

/* Creates a context on HIP device `device` using `hip_stream` (a hipStream_t,
 * may be NULL for the null stream).  *out receives the context. */
int ts_create(ts_ctx** out, int device, void* hip_stream);

/* Frees the context and its workspace.  NULL is accepted. */
int ts_destroy(ts_ctx* ctx);

/* Message of the last error on this context (never NULL). */
const char* ts_last_error(const ts_ctx* ctx);

/* Persistence diagram D(f) (Sec. 2.2): the pairs with v_birth != v_death and
 * the essential class at (f(v_min), f(v_max)), in diagram order (Sec. 2.4):
 * by rank of v_birth, then rank of v_death, dim, and the birth simplex's
 * lexicographic key.
 *   f:        n floats, device or host (on_device)
 *   out:      host array of `capacity` records
 *   n_out:    receives |D(f)|; TS_ERR_CAPACITY if it exceeds capacity */
int ts_diagram(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
               ts_pair* out, int64_t capacity, int64_t* n_out);

/* Persistence diagrams of a batch of fields of different sizes (Sec. 2.2),
 * computed together: the fields are copied one after another into one device
 * buffer and every stage of the persistence map runs once over the whole
 * batch.  Field i's diagram is exactly ts_diagram of field i alone (same
 * records, same order, ids local to the field).
 *   nf:       number of fields (>= 1); the batch holds at most 2^25 vertices
 *   f:        host array of nf field pointers, each device or host (on_device)
 *   dims:     host array of 3 * nf sizes (Lx, Ly, Lz of each field, each >= 2)
 *   out:      host array of `capacity` records: field 0's diagram, then field 1's, ...
 *   counts:   host array of nf entries, receives |D(f_i)| (also when the total
 *             exceeds capacity, which returns TS_ERR_CAPACITY) */
int ts_diagram_batch(ts_ctx* ctx, int32_t nf, const float* const* f, const int64_t* dims,
                     int32_t on_device, ts_pair* out, int64_t capacity, int64_t* counts);

/* Topological simplification (Alg. 1 with Sec. 4.1 and 4.3).
 *   f:  n floats (input, never modified), device or host (opt->inputs_on_device)
 *   g:  n floats (output), same memory kind as f, must not overlap f
 *   rep: receives the report
 * Returns TS_OK when the stop rule held, TS_WARN_NOT_CANCELLED when j_max
 * was reached first, or an error. */
int ts_simplify(ts_ctx* ctx, const float* f, const int64_t dims[3], const ts_signal* sig,
                const ts_options* opt, float* g, ts_report* rep);

/* Topological simplification of a batch of fields of different sizes
 * (Alg. 1 per field).  The persistence maps of all fields run together, every
 * stage one launch over the batch; the update step runs once for all fields
 * still running.  Each field keeps its own targets (threshold relative to its
 * own range), still join, assignment and stop rule, and a field stops being
 * updated once its rule holds: g[i] and reps[i] (iterations, losses, sizes)
 * are those of ts_simplify on field i alone.  The time fields and
 * n_regradient of every report are those of the whole batch.
 *   nf:   number of fields (>= 1); the batch holds at most 2^25 vertices
 *   f, g: host arrays of nf pointers (device or host per opt->inputs_on_device);
 *         no g[i] may overlap an f[k] or another g[k]
 *   dims: host array of 3 * nf sizes
 *   sig:  mode 0 (persistence threshold) only
 *   reps: host array of nf reports
 * Returns TS_OK when every field's stop rule held, TS_WARN_NOT_CANCELLED
 * otherwise, or an error. */
int ts_simplify_batch(ts_ctx* ctx, int32_t nf, const float* const* f, const int64_t* dims,
                      const ts_signal* sig, const ts_options* opt, float* const* g,
                      ts_report* reps);

/* Signal-vertex mask of D(f) (Sec. 3): mask[v] = 1 at the birth and death
 * vertices of every pair that `sig` keeps as signal (the rule ts_simplify
 * applies to D(f0): threshold relative to max f - min f, or the explicit
 * list; the essential pair always counts), 0 elsewhere.  This is the second
 * input channel of the warm-start network.
 *   f:        n floats, device or host (on_device)
 *   mask:     n floats (output), same memory kind as f, must not overlap f
 *   n_signal: receives the number of signal pairs (may be NULL) */
int ts_signal_mask(ts_ctx* ctx, const float* f, const int64_t dims[3], const ts_signal* sig,
                   int32_t on_device, float* mask, int64_t* n_signal);

/* ---- the learned warm start ---------------------------------------------
 * A 3D U-Net (3 levels of 16/32/64 channels, two 3x3x3 convolutions with ReLU
 * per level, 2x2x2 average pooling, nearest 2x upsampling with skip
 * concatenation, a 1x1x1 head) maps (field normalised to [0, 1] by its range,
 * signal-vertex mask) to a proposed change (g0 - f) / range.  It is not part
 * of the paper's method: a start point g0 for the exact solver, which still
 * decides every result (ts_options.init).  Convolutions run on BF16 MFMA
 * tiles with FP32 accumulation; activations are BF16, parameters FP32.
 * Volumes are channels-last, voxel v = x + Lx * (y + Ly * z); each size a
 * multiple of 4.  Every pointer below is a device pointer. */

/* Number of FP32 parameters: per convolution [27][Cout][Cin] weights and
 * Cout biases (layers 8->16 (input channels 2..7 unused), 16->16, 16->32,
 * 32->32, 32->64, 64->64, 96->32, 32->32, 48->16, 16->16), then the head's 16
 * weights and bias.  No context, no GPU. */
int ts_unet_param_count(int64_t* n);

/* out[v] (V floats) = network(input), input [V][2] floats. */
int ts_unet_forward(ts_ctx* ctx, const float* params, const float* input, const int64_t dims[3],
                    float* out);

/* Forward pass, mean squared error against target [V] (*loss, host), and the
 * gradient of that loss with respect to every parameter (grad, overwritten). */
int ts_unet_backward(ts_ctx* ctx, const float* params, const float* input, const float* target,
                     const int64_t dims[3], float* grad, double* loss);

/* One Adam step on n parameters (m, v: moment buffers, zero at step 1). */
int ts_unet_adam(ts_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t n,
                 int64_t step, float lr, float beta1, float beta2, float eps);

/* ---- stage entry points (for per-stage checks and profiling) ----------- */

/* Vertex order: order[i] = i-th lowest vertex, rank[order[i]] = i.
 * f, order, rank: n entries each, device or host (on_device). */
int ts_order(ts_ctx* ctx, const float* f, int64_t n, int32_t on_device, int32_t* order,
             int32_t* rank);

/* Discrete gradient (Sec. 4.2) as dense partner arrays over canonical ids
 * (host arrays): vup[v] = edge paired with vertex v, eup[e] = triangle paired
 * with edge e, tup[t] = tetrahedron paired with triangle t; -1 when the cell
 * is not paired with a coface, -2 when the id is not a cell of the grid.
 * Sizes n, 7n, 12n. */
int ts_gradient(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
                int32_t* vup, int32_t* eup, int32_t* tup);

/* Critical cells sorted by (dim, lexicographic key): host arrays out_dim,
 * out_id of `capacity` entries; counts[4] receives the per-dim counts. */
int ts_critical(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
                int32_t* out_dim, int64_t* out_id, int64_t capacity, int64_t counts[4]);

/* All pairs of the critical cells, including zero-persistence ones, plus the
 * essential class, sorted by (dim, birth_cell, death_cell); host output. */
int ts_pairs(ts_ctx* ctx, const float* f, const int64_t dims[3], int32_t on_device,
             ts_pair* out, int64_t capacity, int64_t* n_out);

/* W2^2 assignment of one dimension (Eq. 1 with q = 2 on the augmented
 * diagrams, Sec. 2.3 and 4.3), as used by ts_simplify for the pairs that are
 * not still.  Host arrays: points (pb[i], pd[i]), targets (qb[j], qd[j]);
 * match[i] receives the target index or -1 (diagonal); *cost the total
 * (matched squared distances + diagonal costs of everything else).
 * A point and a target with c(p,q) >= diag(p) + diag(q) are never matched.
 * The result is the exact optimum: after exact reductions, a problem of at
 * most 1000 points + targets is solved by successive shortest paths; a
 * larger one by an epsilon-scaled forward/reverse auction (final eps
 * 1e-10 * W, W = max diag(p) + max diag(q)) whose result is then proved
 * optimal by complementary slackness with exact duals (up to 4 ulps of the
 * terms compared), trading along cost-reducing cycles where it is not.
 * TS_ERR_INTERNAL if no certificate is reached.
 * Needs no context and no GPU. */
int ts_assign(int64_t n_pts, const double* pb, const double* pd, int64_t n_tgt, const double* qb,
              const double* qd, int32_t* match, double* cost);

/* The same problem by the epsilon-scaled auction alone, as ts_simplify runs it
 * with assign_precision = rel_precision (Sec. 5 uses 0.01): the returned total
 * is at most (1 + rel_precision)^2 times the optimum.  rel_precision = 0 gives
 * the exact assignment of ts_assign.  Host arrays as in ts_assign;
 * TS_ERR_ARG for a negative or non-finite rel_precision.  Needs no context
 * and no GPU. */
int ts_assign_auction(int64_t n_pts, const double* pb, const double* pd, int64_t n_tgt,
                      const double* qb, const double* qd, double rel_precision, int32_t* match,
                      double* cost);

/* Vertex order (as ts_order) for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It needs no context and allocates nothing: its temporaries
 * (sort keys and values with their ping-pong buffers, digit histograms, scan
 * sums, a flag) live in one static device array of 2^21 * 16 bytes + 1 MiB
 * (33 MiB), which every device that runs this call holds until the process
 * ends.  Calls that overlap on one device share that array and race: order
 * them on one stream.
 *   f:      n floats, device pointer on the current device
 *   n:      1 .. 2^21 (2,097,152); larger sizes return TS_ERR_ARG
 *   order, rank: n int32 each, device pointers; no two of f, order, rank
 *           may overlap
 *   hip_stream: the hipStream_t to run on (NULL: the null stream); the call
 *           waits for it before returning (it reads back the non-finite flag)
 * Returns TS_OK, TS_ERR_ARG, TS_ERR_NONFINITE (NaN or Inf in f), TS_ERR_HIP. */
int ts_order_noalloc(const float* f, int64_t n, int32_t* order, int32_t* rank, void* hip_stream);

/* Per-kernel device time (ms) of the last ts_diagram / ts_simplify call,
 * measured with HIP events on the context's stream: stage_ms[i] for the
 * stage named stage_names[i] (NULL-terminated list).  Returns the count. */
int ts_stage_times(const ts_ctx* ctx, const char* const** names, const double** ms);

/* The launch tuner's choices so far.  Some launch shapes are picked by timing
 * each candidate once on the first calls of a size class (the results do not
 * depend on the choice); keys[i] names the launch and its size class
 * (floor(log2 size) + 1), choices[i] is the index of the candidate in use,
 * or -1 while candidates are still being tried:
 *   "k3.tiles.<c>", "k3.tiles.batch.<c>" (c from the vertex count): tile
 *       shape of the lower-star gradient, 0..5 = 256x1x1, 64x4x1, 32x8x1,
 *       32x4x2, 16x4x4, 8x8x4 vertices, 6 = runs of 256 consecutive vertex
 *       ids;
 *   "d1.block.<c>" (c from the column count): block of the saddle-saddle
 *       reduction, 0..4 = 2^16, 2^17, 2^18, 2^20, 2^24 columns.
 * The arrays stay valid until the next call on ctx; keys is NULL-terminated.
 * Returns the count, or TS_ERR_ARG. */
int ts_launch_choices(ts_ctx* ctx, const char* const** keys, const int** choices);

#ifdef __cplusplus
}
#endif
#endif
