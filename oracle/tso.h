/*
 * tso.h -- CPU oracle for scalar-field topological simplification.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the GPU path is checked against.  Only the test
 * suite, the package smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the GPU
 * library; the two agree only on the documented id and record formats.
 *
 * Paper: Kissi, Pont, Levine, Tierny, "A Practical Solver for Scalar Data
 * Topological Simplification" (arXiv 2407.12399).
 *
 * Conventions (formats shared with the GPU library by documentation only):
 *  - Field: float32 [Lz][Ly][Lx], vertex id v = x + Lx*(y + Ly*z).
 *  - Triangulation: Freudenthal/Kuhn (Sec. 2.1).  A cell anchored at vertex u
 *    is {u + c0, ..., u + ck} with 0 = c0 < c1 < ... < ck <= (1,1,1) a chain
 *    of unit-cube corners (corner mask bit0 = x, bit1 = y, bit2 = z).
 *    Canonical ids: edge 7u+t, triangle 12u+t, tetrahedron 6u+t with types
 *      edge t:      c1 = t+1
 *      triangle t:  (c1,c2) in (1,3)(2,3)(1,5)(4,5)(2,6)(4,6)
 *                              (1,7)(2,7)(3,7)(4,7)(5,7)(6,7)
 *      tet t:       (c1,c2,7) with (c1,c2) in (1,3)(1,5)(2,3)(2,6)(4,5)(4,6)
 *    A cell id is valid iff u + ck lies inside the grid.
 *  - Vertex order: (value, id) ascending with -0.0 taken as +0.0 (Sec. 2.1,
 *    simulation of simplicity).  rank[v] = position of v in that order.
 *  - Lexicographic filtration (Sec. 2.2): a cell's key is the ranks of its
 *    vertices sorted decreasingly; keys compare lexicographically, a proper
 *    prefix first.
 *
 * Every function returns 0 on success and a negative code on error:
 *   -1 bad argument, -2 non-finite input, -5 output capacity too small
 *   (the required size is still written to *n_out).
 */
#ifndef TSO_H
#define TSO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One persistence pair (Sec. 2.2).  48 bytes. */
typedef struct {
  int32_t dim;        /* 0 min-saddle, 1 saddle-saddle, 2 saddle-max */
  int32_t essential;  /* 1: infinite class, death_cell = -1, v_death = v_max */
  int64_t birth_cell; /* canonical id of the birth simplex (dim `dim`) */
  int64_t death_cell; /* canonical id of the death simplex (dim `dim`+1) */
  int64_t v_birth;    /* highest vertex of the birth simplex */
  int64_t v_death;    /* highest vertex of the death simplex */
  float birth;        /* f(v_birth) */
  float death;        /* f(v_death) */
} tso_pair;

/* Signal selection (Sec. 3). */
typedef struct {
  int32_t mode;                /* 0: persistence threshold, 1: explicit list */
  float threshold_rel;         /* threshold = threshold_rel * range(f0) */
  uint32_t nonsignal_dim_mask; /* bit k: dim-k pairs below threshold are non-signal */
  int32_t ties_signal;         /* persistence == threshold: 1 signal, 0 non-signal */
  const tso_pair* signal;      /* mode 1: signal pairs, matched on (dim, birth_cell, death_cell) */
  int64_t n_signal;
} tso_signal;

/* Solver options (Sec. 4.1, Sec. 5). */
typedef struct {
  float alpha_b, alpha_d;  /* gradient step sizes, paper default 0.5 / 0.5 */
  int32_t j_max;           /* maximum iterations, paper default 1000 */
  int32_t stop_mode;       /* 0: all non-signal persistence < cancel_tol_rel*range,
                              1: loss <= loss_ratio_s * loss0 (Alg. 1) */
  float cancel_tol_rel;    /* 1e-6 */
  float loss_ratio_s;      /* 0.01 */
} tso_options;

typedef struct {
  int32_t iterations;      /* gradient steps performed */
  int32_t cancelled;       /* 1 if the stop rule was met before j_max */
  double loss0, loss;      /* L at iteration 0 and at the end (sum over diagram points) */
  double energy;           /* loss + diagonal cost of unmatched targets */
  double linf, l2;         /* ||f-g||_inf, ||f-g||_2 */
  double max_nonsignal_pers; /* max persistence among diagonal-assigned points */
  double max_signal_disp;  /* max distance of a target-assigned point to its target */
  double range;            /* max(f0) - min(f0) */
  int64_t n_pairs[3];      /* final diagram size per dimension (finite pairs) */
  int64_t n_still;         /* still pairs at the last iteration */
  int64_t n_reduced;       /* reduced-problem points at the last iteration */
  int64_t n_targets;       /* |D_T| */
  double total_s;          /* wall time */
} tso_report;

/* Vertex order (Sec. 2.2): order[i] = i-th lowest vertex, rank[order[i]] = i. */
int tso_order(const float* f, int64_t n, int32_t* order, int32_t* rank);

/* Discrete gradient (Sec. 4.2, lower-star algorithm of Robins et al.) as dense
 * partner arrays over canonical ids: vup[v] = edge paired with vertex v,
 * eup[e] = triangle paired with edge e, tup[t] = tetrahedron paired with
 * triangle t; -1 = not paired with a coface, -2 = id is not a valid cell.
 * Arrays have n, 7n and 12n entries. */
int tso_gradient(const float* f, const int64_t dims[3], int32_t* vup,
                 int32_t* eup, int32_t* tup);

/* Lower-star gradient of one vertex, from a rank array.  Writes the pairs
 * (face dim, face id, coface id) and the critical cells (dim, id) of L(v),
 * each list sorted by (dim, id).  Capacities: 74 pairs, 75 critical cells. */
int tso_gradient_at(const int32_t* rank, const int64_t dims[3], int64_t v,
                    int32_t* pair_dim, int64_t* pair_face, int64_t* pair_coface,
                    int32_t* n_pairs, int32_t* crit_dim, int64_t* crit_id,
                    int32_t* n_crit);

/* Critical cells (Sec. 4.2) sorted by (dim, lexicographic key). */
int tso_critical(const float* f, const int64_t dims[3], int32_t* out_dim,
                 int64_t* out_id, int64_t capacity, int64_t* n_out);

/* All persistence pairs, including zero-persistence ones, plus the one
 * essential class; sorted by (dim, birth_cell, death_cell).
 *   method 0: discrete-gradient pairing restricted to critical cells
 *             (union-find for dims 0 and 2, Morse-boundary reduction for dim 1)
 *   method 1: full boundary-matrix reduction of the whole filtered complex
 *             (definition; tiny grids only)
 *   method 2: Kruskal over all edges (dim 0) and dual Kruskal over all
 *             triangles (dim 2); dim-1 pairs are not produced. */
int tso_pairs(const float* f, const int64_t dims[3], int32_t method,
              tso_pair* out, int64_t capacity, int64_t* n_out);

/* Persistence diagram D(f) (Sec. 2.2): pairs with v_birth != v_death plus the
 * essential class at (f(v_min), f(v_max)), in diagram order (rank v_birth,
 * rank v_death, dim, birth-cell key). */
int tso_diagram(const float* f, const int64_t dims[3], tso_pair* out,
                int64_t capacity, int64_t* n_out);

/* Exact W2^2 assignment of one dimension (Eq. 1 with q = 2, Sec. 4.1):
 * points (pb,pd) against targets (qb,qd) with the diagonal available to both.
 * match[i] = target index or -1 (diagonal).  *cost = optimal total cost.
 * Pairs with c(p,q) >= diag(p)+diag(q) are not allowed (ties go to the
 * diagonal). */
int tso_assign(int64_t n_pts, const double* pb, const double* pd,
               int64_t n_tgt, const double* qb, const double* qd,
               int32_t* match, double* cost);

/* One assignment step of the solver (Sec. 4.3, with Eq. (1) on the reduced
 * problem), exactly as tso_simplify runs it at iteration j >= 1:
 *   prev[n_prev], phi_prev: D(f_{j-1}) in diagram order and its assignment
 *                           (target index or -1 for the diagonal);
 *   cur[n_cur]:             D(f_j) in diagram order;
 *   targets[n_tgt]:         D_T (v_birth, v_death = the vertices in D(f0);
 *                           birth, death = the target coordinates; at most
 *                           one essential entry);
 *   phi_out[n_cur]:         receives the assignment of D(f_j).
 * Still points (same (dim, v_birth, v_death) as a point of prev, the k-th
 * occurrence of a key matched with the k-th) keep phi_prev; the essential
 * point always takes the essential target; the other points are assigned
 * exactly, per dimension, to the targets that no still point holds, then
 * put in canonical form.  *n_still, *n_reduced receive the counts. */
int tso_assign_step(const tso_pair* prev, int64_t n_prev, const int32_t* phi_prev,
                    const tso_pair* cur, int64_t n_cur, const tso_pair* targets,
                    int64_t n_tgt, int32_t* phi_out, int64_t* n_still, int64_t* n_reduced);

/* Threads the gradient (Sec. 4.2) and vertex-order loops use: 1 for the
 * checker; the OpenMP timing build (same source, -fopenmp) reports its
 * thread count. */
int tso_threads(void);

/* Bottleneck distance (L-infinity ground metric) between two diagrams;
 * finite points of equal dimension and the essential classes are matched
 * separately.  Small inputs only. */
int tso_bottleneck(const tso_pair* a, int64_t na, const tso_pair* b,
                   int64_t nb, double* out);

/* Topological simplification (Alg. 1 with the direct gradient step of Sec. 4.1
 * and the still-pair assignment reuse of Sec. 4.3).  g receives n floats.
 * Optional per-iteration trace: if trace != NULL, trace[j] = loss after
 * iteration j (j = 0..iterations), up to trace_cap entries. */
int tso_simplify(const float* f, const int64_t dims[3], const tso_signal* sig,
                 const tso_options* opt, float* g, tso_report* rep,
                 double* trace, int64_t trace_cap);

#ifdef __cplusplus
}
#endif
#endif
