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

// Every eigenpair of matrices of at most kHouseholderMaxM columns with no
// host step in between (Householder reduction, tridiagonal eigenpairs,
// back-transformation; the same kernels as a full wide_eigh run), for
// batches whose launch sequence must not wait on the host.  The caller lays
// out, per matrix, hh_scratch_bytes(m) of device scratch and hh_node_bytes()
// of descriptor (uploaded with its other descriptors), then launches them all
// with hh_launch.  Per matrix the finishing kernel writes
//   *floor_out = max(-lambda_min, 0, u_p trace(G) / 10)   (the truncation's
//   rounding level, as a full run reports it), and
//   diag_out[0] = trace(G), diag_out[1] = sum of the eigenvalues.
constexpr int64_t kHouseholderMaxM = 256;
// false when HAPOD_FULL_LANCZOS=1 keeps full runs on the Krylov iteration
bool hh_available();
size_t hh_scratch_bytes(int64_t m);
size_t hh_node_bytes();
// Fills the host image of one matrix's descriptor (node, hh_node_bytes()) and
// of its back-transformation lift (LiftNode, all m columns): scratch is the
// matrix's device scratch.
void hh_describe(int64_t m, const double* G, int64_t ldg, double* lambda, double* V, int64_t ldv, char* scratch,
                 double u_p, double* floor_out, double* diag_out, void* node, LiftNode* lift);
// d_nodes: nn descriptors (hh_node_bytes() apart); d_lifts: their nn lift
// descriptors, item bases already set (lift_items in all, 128 x 128 tiles).
hapod_status hh_launch(const void* d_nodes, int nn, int64_t m_max, const LiftNode* d_lifts, int lift_items,
                       hipStream_t stream);

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
