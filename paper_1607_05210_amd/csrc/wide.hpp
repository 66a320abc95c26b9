// Eigensolver for Gram matrices too large for the one-workgroup Jacobi
// kernel: the leading part of the spectrum by a Krylov method on the GPU.
#pragma once

#include <vector>

#include "internal.hpp"

namespace hapod {

struct WideResult {
  int32_t iterations = 0;   // Krylov steps taken
  int32_t block = 0;        // number of eigenpairs computed
  double floor_abs = 0.0;   // rounding level of the Gram's spectrum
  bool exhausted = false;   // the Krylov space took in the whole spectrum above
                            // the rounding level (stopping test met, or k = m)
  double missing = 0.0;     // sum of the Ritz values past the converged block
                            // that lie above both floor_abs and the final
                            // residual norm (energy the block misses)
  double unresolved = 0.0;  // trace(G) minus the block's eigenvalues: energy no
                            // returned pair holds (a multiplicity the Krylov
                            // space never saw shows up here)
  double trace = 0.0;       // trace(G)
  double noise = 0.0;       // level below which a Ritz value is not resolved:
                            // each eigenvalue past the block is at most this
};

typedef void* (*wide_alloc_fn)(void* ctx, size_t bytes);
typedef void (*wide_free_fn)(void* ctx, void* p);

// G: m x m (ld ldg), symmetric, read only.  Writes lambda[0..m) (descending;
// entries beyond the computed block are 0) and the first `block` columns of
// V (m x ?, ld ldv).  u_p: unit roundoff of the precision the Gram was
// formed in.
// full: run all m steps (m <= 768) and return every eigenpair, as a dense
// eigensolver would; else stop once the residuals reach the rounding level.
hapod_status wide_eigh(const double* G, int64_t ldg, int64_t m, double* lambda, double* V, int64_t ldv,
                       double u_p, wide_alloc_fn alloc, wide_free_fn release, void* ctx, hipStream_t stream,
                       WideResult* res, bool full = false);
constexpr int kWideMaxSteps = 768;

// Several matrices at once (same results as one call each): every step of
// the iteration is one launch per kernel for all matrices still iterating.
struct WideJob {
  const double* G;
  int64_t ldg;
  int64_t m;
  double* lambda;
  double* V;
  int64_t ldv;
  bool full;
  WideResult* res;
};
hapod_status wide_eigh_batch(std::vector<WideJob>& jobs, double u_p, wide_alloc_fn alloc, wide_free_fn release,
                             void* ctx, hipStream_t stream);

}  // namespace hapod
