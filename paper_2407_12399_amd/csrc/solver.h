// solver.h -- simplification loop (Alg. 1 with Sec. 4.1 and Sec. 4.3).
#pragma once

#include <vector>

#include "internal.h"

namespace ts {

Grid make_grid(const int64_t dims[3]);

// Runs the solver; f and g are device pointers when opt.inputs_on_device.
int simplify(ts_ctx* ctx, const float* f, const Grid& grid, const ts_signal& sig,
             const ts_options& opt, float* g, ts_report* rep);

// Signal-vertex mask (Sec. 3): mask[v] = 1 at the birth and death vertices of
// the pairs of D(f) that the signal rule keeps (the rule ts_simplify applies
// to D(f0)), 0 elsewhere.  mask is a device pointer when on_device.  Returns
// the number of signal pairs.
int64_t signal_mask(ts_ctx* ctx, const float* f_dev, const Grid& grid, const ts_signal& sig,
                    float* mask, int on_device);

struct Batch;

// The solver on a batch of fields (f[i], g[i], reps[i] per field): the
// persistence maps of all fields run together, each field keeps its own
// solve (the result of each field is that of simplify on it alone).
int simplify_batch(ts_ctx* ctx, const Batch& B, const float* const* f, const ts_signal& sig,
                   const ts_options& opt, float* const* g, ts_report* reps);

// Exact W2^2 assignment of one dimension on the augmented diagrams
// (Eq. 1, q = 2): match[i] = target index or -1 (diagonal).  Pairs with
// c(p,q) >= diag(p) + diag(q) are excluded.  Returns the optimal cost.
double assign_exact(const std::vector<double>& pb, const std::vector<double>& pd,
                    const std::vector<double>& qb, const std::vector<double>& qd,
                    std::vector<int>* match);

// The same problem by an epsilon-scaled auction to eps_rel * W, W = max
// diag(p) + max diag(q).  With gap_rel == 0 its result is then proved optimal
// (complementary slackness with exact duals, trading along cost-reducing
// cycles where it is not), so the return is the exact optimum; if the
// certificate's work budget runs out it throws CertificateMissing.  With
// gap_rel > 0 it stops after the first phase whose total is within
// (1 + gap_rel)^2 of the dual lower bound, with no certificate.
double assign_auction(const std::vector<double>& pb, const std::vector<double>& pd,
                      const std::vector<double>& qb, const std::vector<double>& qd,
                      std::vector<int>* match, double eps_rel, double gap_rel = 0.0);

// The solver's choice: exact reductions, then successive shortest paths up
// to a problem size and the certified auction above it (both exact); with
// gap_rel > 0 the auction with that stopping gap for every size.
double assign_reduced(const std::vector<double>& pb, const std::vector<double>& pd,
                      const std::vector<double>& qb, const std::vector<double>& qd,
                      std::vector<int>* match, double gap_rel = 0.0,
                      bool auction_only = false);

}  // namespace ts
