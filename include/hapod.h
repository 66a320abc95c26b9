/*
 * hapod.h -- C ABI of the MI355X (gfx950) hierarchical approximate POD.
 *
 * The library computes, for every node of a rooted tree, the local POD of the
 * node's input columns by the method of snapshots (Rem. 2.3 of Himpe, Leibner
 * & Rave, "Hierarchical Approximate POD"):
 *
 *   Gram      G = S^T S                                   (Rem. 2.3)
 *   eigh      G = V diag(lambda) V^T, lambda descending   (Rem. 2.3)
 *   truncate  N = min{N' : sum_{n>N'} lambda_n <= eps^2}   (Def. 2.5, Thm. 2.4)
 *   lift      inner node: W = S V_N          (= U Sigma, the scaled modes)
 *             root:       U = S V_N Lambda_N^(-1/2)       (Rem. 2.3, Def. 3.2)
 *
 * and drives those node PODs level by level over the tree (Def. 3.1, Def. 3.2)
 * with the local tolerances of Thm. 3.5.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major with a leading dimension ("ld") >= rows.
 * - Snapshot / mode storage type follows the precision: HAPOD_FP64 stores
 *   double, HAPOD_FP32 and HAPOD_BF16X3 store float.  Gram matrices,
 *   eigenvalues, eigenvectors, singular values and tolerances are always
 *   double.
 * - "device" pointers are HIP device allocations on the current device;
 *   "host" pointers are ordinary host memory.  Each argument says which.
 * - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *   device work is ordered on it.  Entry points that return host results
 *   synchronise the stream before returning; the others are asynchronous.
 * - The caller owns every buffer it passes in.  The library never frees
 *   caller memory and never keeps a caller pointer beyond the call, except
 *   leaf pointers returned by a leaf provider, which must stay valid until
 *   hapod_run returns.
 * - Every function returns a status and never aborts; a human-readable
 *   message for the last failure on the calling thread is returned by
 *   hapod_last_error().
 * - Results are deterministic: reductions run in a fixed order and no
 *   floating-point atomics are used, so reruns are bitwise identical.
 */
#ifndef HAPOD_H
#define HAPOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HAPOD_OK = 0,
  HAPOD_E_INVALID = 1,   /* bad argument (negative size, eps < 0, omega outside [0,1], NULL) */
  HAPOD_E_TREE = 2,      /* parent array violates Def. 3.1 (roots, range, cycles)           */
  HAPOD_E_NOMEM = 3,     /* device allocation failed or the memory cap would be exceeded    */
  HAPOD_E_DEVICE = 4,    /* a HIP runtime call failed                                       */
  HAPOD_E_NUMERIC = 5,   /* non-finite Gram diagonal (NaN/Inf in the input)                 */
  HAPOD_E_STATE = 6,     /* plan not run yet / node has no result                           */
  HAPOD_E_CALLBACK = 7,  /* the leaf provider returned a non-zero code                      */
  HAPOD_E_UNSUPPORTED = 8 /* size beyond a kernel's documented limit, or a node wider than
                             the Jacobi limit whose Krylov eigensolve (at most 768 steps) did
                             not resolve every eigenvalue its truncation needs             */
} hapod_status;

typedef enum {
  HAPOD_FP64 = 0,    /* Gram and lift on FP64 MFMA, double storage                         */
  HAPOD_FP32 = 1,    /* Gram and lift on FP32 MFMA, FP32 accumulation, float storage       */
  HAPOD_BF16X3 = 2   /* float storage; Gram of nodes of more than 64 columns as split-BF16,
                        three products hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32
                        accumulation; narrower Grams and all lifts on FP32 MFMA        */
} hapod_precision;

/* ------------------------------------------------------------------------ */
/* Step-level entry points: one method-of-snapshots step each.              */
/* ------------------------------------------------------------------------ */

/* Gram matrix G = S^T S (Rem. 2.3).
 *   S      device, n x m column-major, ld lds >= n, storage type of prec.
 *   G      device, m x m double, ld ldg >= m; the full symmetric matrix is
 *          written (both triangles, bitwise symmetric).
 * Row blocks are accumulated in the precision's MFMA accumulator and the
 * block partial sums are added in double, in a fixed order.
 * n == 0 gives G = 0; m == 0 is a no-op.                                    */
hapod_status hapod_gram(hapod_precision prec, int64_t n, int64_t m,
                        const void* S, int64_t lds, double* G, int64_t ldg,
                        void* stream);

/* hapod_gram for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same G = S^T S, with the same arguments and results, computed without any
 * allocation or host staging.  Descriptors and partial tiles live in a
 * library-owned device array of 64.25 MiB per device (held until the process
 * ends); its device address is looked up on the first call on each device.
 * m <= 256 (HAPOD_E_UNSUPPORTED above); the row chunks are capped at 128, so
 * the sums may be ordered differently from hapod_gram's (equal within the
 * same rounding bound; bitwise equal on exactly representable data).
 * Asynchronous: nothing is synchronised or copied to the host.  Calls on one
 * device share the array: calls that overlap on one device (other streams,
 * other threads) race and must not be made.                                */
hapod_status hapod_gram_noalloc(hapod_precision prec, int64_t n, int64_t m,
                                const void* S, int64_t lds, double* G, int64_t ldg,
                                void* stream);

/* Symmetric eigendecomposition of a Gram matrix (Rem. 2.3), in double.
 *   G       device, m x m, ld ldg; overwritten (destroyed).
 *   lambda  device, m doubles: eigenvalues, descending; equal values keep
 *           their original index order.
 *   V       device, m x m double, ld ldv: orthonormal eigenvectors, column k
 *           for lambda[k], each with its largest-magnitude entry positive.
 *   sweeps  host, may be NULL: Jacobi sweeps used.
 * Synchronises the stream when sweeps != NULL.  m <= HAPOD_EIG_MAX.         */
#define HAPOD_EIG_MAX 8192
hapod_status hapod_eigh(int64_t m, double* G, int64_t ldg, double* lambda,
                        double* V, int64_t ldv, int32_t* sweeps, void* stream);

/* Truncation rank of Def. 2.5 from eigenvalues of a Gram matrix.
 *   lambda  device, m doubles, descending.  Negative values are rounding
 *           artefacts of the Gram product; they count as zero energy.
 *   eps     the local tolerance; the rank is the smallest N with
 *           sum_{n>N} max(lambda_n, 0) <= eps^2 (tail summed in double).
 *   info    host, 4 doubles, may be NULL: {tail(N), lambda_1, lambda_min,
 *           number of negative eigenvalues}.
 *   rank    host.
 * Synchronises the stream.                                                  */
hapod_status hapod_truncate(int64_t m, const double* lambda, double eps,
                            int64_t* rank, double* info, void* stream);

/* Mode lift (Rem. 2.3, Def. 3.2).
 *   S       device, n x m, ld lds, storage type of prec.
 *   V       device, m x N double, ld ldv (eigenvectors for the kept modes).
 *   lambda  device, N doubles, or NULL.  NULL: out = S V (scaled modes
 *           sigma_k phi_k, what a parent node consumes).  Non-NULL:
 *           out = S V diag(lambda)^(-1/2) (orthonormal modes, the root's
 *           output).
 *   out     device, n x N, ld ldo, storage type of prec.
 * Products: FP64 MFMA (HAPOD_FP64), FP32 MFMA (HAPOD_FP32), three BF16
 * products per term with FP32 accumulation (HAPOD_BF16X3).                 */
hapod_status hapod_lift(hapod_precision prec, int64_t n, int64_t m, int64_t N,
                        const void* S, int64_t lds, const double* V, int64_t ldv,
                        const double* lambda, void* out, int64_t ldo,
                        void* stream);

/* Re-orthonormalisation of computed modes in double: two passes of
 * Cholesky-QR (W = U^T U accumulated in double, W = R^T R, U <- U R^-1).
 *   U  device, n x N, ld ldu, storage type of prec; overwritten.
 * Columns whose Cholesky pivot is not positive are left as they are and
 * reported through *bad (host, may be NULL).  N <= 1024.                    */
hapod_status hapod_reorth(hapod_precision prec, int64_t n, int64_t N, void* U,
                          int64_t ldu, int64_t* bad, void* stream);

/* One local POD(S, eps) (Def. 2.5) by the method of snapshots.
 *   S       device, n x m, ld lds, storage type of prec.
 *   eps     >= 0.  eps == 0 is the pass-through POD(S, 0) = {(1, s)}: out
 *           receives a copy of S and every sigma is 1 (Def. 2.5).
 *   scaled  0: out holds orthonormal modes phi_k; 1: out holds sigma_k phi_k.
 *   out     device, n x m capacity, ld ldo, storage type of prec; the first
 *           *rank columns are written.
 *   sigma   host, m doubles capacity; the first *rank are written.
 *   rank    host.
 * Synchronises the stream.                                                  */
hapod_status hapod_node_pod(hapod_precision prec, int64_t n, int64_t m,
                            const void* S, int64_t lds, double eps, int32_t scaled,
                            void* out, int64_t ldo, double* sigma, int64_t* rank,
                            void* stream);

/* One local POD(S, eps) (Def. 2.5) without the method of snapshots' Gram
 * eigenproblem, whose squared condition number (Rem. 2.3) limits the
 * singular values to about sqrt(u) sigma_1 (absolute): S = Q R by
 * Cholesky-QR passes Q <- Q R_p^-1, each shifted (Q^T Q + s I = R_p^T R_p
 * with s = 11 (n m + m (m + 1)) u trace(Q^T Q), Fukaya et al., SIAM J. Sci.
 * Comput. 2020) while m max|Q^T Q - I| > 1/2, until two plain passes
 * follow each other, the first on the column-equilibrated Gram (columns of
 * any size start on equal terms; a column with a zero Gram diagonal gives
 * singular value 0); the SVD R V = U_R diag(sigma) by one-sided Jacobi;
 * the modes Q U_R.  The sigma_k are accurate to about u sigma_1,
 * rank-deficient S included.
 * FP64 only; m <= 512 and m <= n (HAPOD_E_UNSUPPORTED otherwise, eps > 0).
 *   S, lds, eps, scaled, out, ldo, sigma, rank   as hapod_node_pod (double).
 *   passes  host, may be NULL: Cholesky-QR passes taken (3 for a
 *           well-conditioned S, up to about 7 at condition 1e14 or rank
 *           loss).
 *   sweeps  host, may be NULL: Jacobi sweeps taken.
 * HAPOD_E_NUMERIC: a pivot was not positive (non-finite input), or no
 * orthonormal Q in 12 passes, or no Jacobi convergence in 60 sweeps.
 * Scratch: two n x m double buffers and a few m x m ones from the library's
 * pool.  Synchronises the stream (twice per pass).                         */
hapod_status hapod_node_pod_qr(int64_t n, int64_t m, const double* S, int64_t lds,
                               double eps, int32_t scaled, double* out, int64_t ldo,
                               double* sigma, int64_t* rank, int32_t* passes,
                               int32_t* sweeps, void* stream);

/* One local POD(S, eps) (Def. 2.5) of a wide S (many more columns than its
 * rank) by a randomized range finder (Halko, Martinsson & Tropp, SIAM Review
 * 2011), without the Gram eigenproblem whose squared condition number
 * (Rem. 2.3) limits the method of snapshots to sigma_k^2 above about
 * u sigma_1^2:
 *   Y = S Omega, Q = orth(Y) by Cholesky-QR passes (as hapod_node_pod_qr),
 *   B = Q^T S, r = ||S - Q B||_F^2 summed from the residual columns
 *   themselves, the SVD of B from the QR factor of B^T (Cholesky-QR passes,
 *   one-sided Jacobi on R'^T), modes Q U_B.
 * Omega (m x ell), from counter-based generators and `seed`:
 *   kind 0: a sparse sign map (Martinsson & Tropp, Acta Numerica 2020,
 *     Sec. 9.2) in block-shifted form: 8 nonzeros +-1/sqrt(8) per row, one
 *     in each of 8 column blocks of bw = ell / 8; per chunk of bw
 *     consecutive rows of Omega and per block, the positions are one cyclic
 *     shift of 0 .. bw - 1 and every position has its own sign, shift and
 *     signs from the splitmix64 finaliser; Y costs one pass over S.  Should
 *     r exceed eps^2, the route starts over with the Gaussian;
 *   kind 1: Gaussian (Box-Muller over the splitmix64 finaliser).
 * Rank: the smallest N with r + sum_{k>N} sigma_k(B)^2 <= eps^2, so the
 * modes' projection error ||S - U U^T S||_F^2 = r + sum_{k>N} sigma_k(B)^2
 * is at most eps^2 (Def. 2.5's requirement, as used by Thm. 3.3 - 3.5).
 * Unscaled modes (scaled = 0) take that error from the modes themselves:
 * N is chosen with eps^2 / 64 of the budget left for r, then
 * ||S - U C||_F^2 with C = U^T S = U_B[:, :N]^T B (an n x m x N product in
 * place of the n x m x ell one for r) must come out <= eps^2; should it
 * not, r is computed and N set exactly as above.  r is then reported as
 * that error less sum_{k>N} sigma_k(B)^2.
 * FP64 only.  ell in {128, 256, 384, 512}, ell <= m, ell <= n
 * (HAPOD_E_UNSUPPORTED otherwise); eps > 0 and kind 0 or 1
 * (HAPOD_E_INVALID otherwise).
 *   S, lds, eps, scaled, out, ldo, sigma, rank   as hapod_node_pod (double);
 *           sigma and out need ell entries / columns of capacity.
 *   info7   host, may be NULL: {r, passes on Y, passes on B^T, Jacobi sweeps,
 *           device ms, ell, the test matrix of the result (0 sparse sign,
 *           1 Gaussian)}.
 * r > eps^2 with the Gaussian (the rank of S within eps exceeds what ell
 * columns capture): HAPOD_E_UNSUPPORTED, info7 still filled.
 * Scratch: two n x ell double buffers, an m x ell Gaussian and B^T, partial
 * sums, from the library's pool.  Synchronises the
 * stream.                                                                  */
hapod_status hapod_node_pod_sketch(int64_t n, int64_t m, const double* S, int64_t lds, double eps,
                                   int32_t scaled, int64_t ell, uint64_t seed, int32_t kind, double* out,
                                   int64_t ldo, double* sigma, int64_t* rank, double* info7, void* stream);

/* ------------------------------------------------------------------------ */
/* Tree-level entry points.                                                 */
/* ------------------------------------------------------------------------ */

typedef struct hapod_plan_s* hapod_plan_t;

/* A rooted tree (Def. 3.1) with the snapshot-to-leaf map D (Def. 3.2):
 *   parent[i]    parent of node i, -1 for the (single) root.
 *   leaf_cols[i] |D^-1(i)|, the number of snapshots at leaf i (ignored for
 *                inner nodes).
 *   n            dimension of the snapshot space V (rows).
 *   leaf_rows    NULL (every leaf holds n rows) or, per node, the number of
 *                leading rows a leaf's snapshots hold (1..n); the remaining
 *                rows are zero and never read.  An inner node's vectors hold
 *                the maximum over its children.
 * Arrays are host memory, read during hapod_plan only.                     */
typedef struct {
  int32_t num_nodes;
  const int32_t* parent;
  const int64_t* leaf_cols;
  int64_t n;
  const int64_t* leaf_rows;
} hapod_tree;

typedef struct {
  hapod_precision prec;
  int32_t reorth;                  /* 1: hapod_reorth on the root modes                    */
  int64_t mem_cap_bytes;           /* 0: no cap; else device bytes the plan may hold       */
  const double* node_eps_override; /* host, num_nodes values or NULL; an entry >= 0
                                      replaces the Thm. 3.5 tolerance of that node         */
  int32_t jacobi_max;              /* k > 0: nodes with at most k input columns (k <= 1024)
                                      take the Jacobi eigensolver, wider ones Lanczos.
                                      0: automatic -- Jacobi up to 64 columns; 65..256
                                      every eigenpair (as Jacobi gives) from a
                                      Householder reduction to tridiagonal form; above
                                      256 Lanczos stopped at the Gram's rounding level */
  int32_t autotune;                /* 1: the first time a node class (precision, width,
                                      height class) is met, time the candidate Gram tiles
                                      on a buffer of its shape and keep the fastest for
                                      the process; 0: fixed tile rule                   */
  int32_t leaf_wave;               /* 0: all leaves of a level in one launch group; k > 0:
                                      at most k leaves per group, so the provider needs at
                                      most k leaves resident at a time                     */
  int32_t block_gram;              /* 1: block-structured Gram at inner nodes -- a computed
                                      child's scaled modes sigma_k u_k have the Gram block
                                      diag(sigma_k^2) (orthonormal u_k), so column-tile
                                      pairs that lie inside one such child's block are not
                                      computed but set to it; the node's raw (pass-through)
                                      columns go first so the children's blocks start on
                                      tile boundaries.  FP64 form only (HAPOD_E_INVALID
                                      otherwise: FP32 modes are not orthonormal enough).
                                      0: every Gram entry computed                      */
  int32_t right_vectors;           /* 1: keep every computed node's right singular vectors
                                      (eigenvectors V[:, :N]) for hapod_right_vectors   */
  int32_t qr_pod;                  /* 1: computed nodes of at most 512 inputs and no more
                                      inputs than rows take the QR route of
                                      hapod_node_pod_qr (their singular values to ~u
                                      sigma_1); the others the method of snapshots.
                                      FP64 only, not with right_vectors
                                      (HAPOD_E_INVALID otherwise).  A QR node's time
                                      counts as Gram time in the phase timings.        */
  int32_t sketch_cols;             /* ell > 0 (128, 256, 384 or 512): computed nodes of at
                                      least 2 ell inputs and ell rows take the sketched
                                      route of hapod_node_pod_sketch with ell sketch
                                      columns (seed fixed per node id), whose truncation
                                      is certified from the residual itself instead of a
                                      Gram spectrum; a node whose rank the sketch cannot
                                      hold fails the run with HAPOD_E_UNSUPPORTED.  FP64
                                      only, not with right_vectors (HAPOD_E_INVALID
                                      otherwise).  0: off.  Timings: sketch, Q, B and
                                      residual count as Gram, the small SVD as
                                      eigensolve, the modes' product as lift.          */
  const char* autotune_cache;      /* path or NULL: with autotune, the tile choices of node
                                      classes are read from this text file when the plan is
                                      made (one line per class: compute mode, width class,
                                      log2 height class, tile) and the process's whole table
                                      written back after every run; the file is replaced
                                      through a temporary one.  Read during
                                      hapod_plan only (the path string is copied).     */
  int32_t graph_levels;            /* 1: each device-driven batch (see
                                      hapod_plan_batch_stats) is captured as a hipGraph
                                      and launched as one; the next run replays the graph
                                      at the same batch position when the batch's
                                      descriptors, device buffers and launch parameters
                                      hash the same (same leaves, same pool blocks), and
                                      captures anew otherwise.  Uploads stay outside the
                                      graph; the phases of a graph-launched batch are not
                                      separated in hapod_run_timing (see
                                      hapod_plan_graph_stats).  0: plain launches.      */
  int32_t sketch_kind;             /* test matrix of the sketched route (sketch_cols):
                                      0: the sparse sign map (see
                                      hapod_node_pod_sketch), the Gaussian if its
                                      residual exceeds eps^2; 1: the Gaussian.  Other
                                      values: HAPOD_E_INVALID.                          */
  int32_t leaf_layout;             /* how a leaf provider's pointer holds the leaf:
                                      0: column-major, leading dimension ld >= rows;
                                      1: this library's row-block layout -- blocks of 128
                                      rows, block b holding rows 128 b .. 128 b + 127 of
                                      every column of the leaf, column j at element
                                      128 j of the block (a block spans 128 x leaf_cols
                                      elements; ld is ignored).  Other values:
                                      HAPOD_E_INVALID.                                   */
  int32_t leaf_passthrough;        /* 1: a computed leaf whose truncation keeps every one
                                      of its columns (rank = leaf_cols, nothing
                                      discarded) hands its own columns to its parent in
                                      place of its scaled modes sigma_k u_k = S v_k: the
                                      same span and Gram spectrum (the right factor V is
                                      orthogonal), so the parent's POD is the same up to
                                      rounding, and the leaf's lift is saved.  Such a
                                      leaf's data is read again when its parent's group
                                      runs (no release call in between; see
                                      hapod_leaf_fn), and its batch reads the ranks back
                                      before the lift.  Not with right_vectors (the leaf
                                      keeps its modes then).  In the FP32 and split-BF16
                                      forms the parent's Gram of the raw columns (nearly
                                      collinear snapshots) loses more to FP32 rounding
                                      than one of orthogonal, graded modes.  0: off.
                                      Other values: HAPOD_E_INVALID.                     */
} hapod_options;

/* Validate the tree (Def. 3.1), compute levels (height: leaves are level 1),
 * |S~_alpha| and the Thm. 3.5 tolerances
 *   eps(root)  = sqrt(|S|) omega eps_star,
 *   eps(alpha) = sqrt(|S~_alpha|) (L_T - 1)^(-1/2) sqrt(1 - omega^2) eps_star,
 * then apply node_eps_override.  opts may be NULL (FP64, no re-orth).
 * No device memory is allocated.                                            */
hapod_status hapod_plan(const hapod_tree* tree, double eps_star, double omega,
                        const hapod_options* opts, hapod_plan_t* out);

/* Host copies of the plan: eps (double), level (int32), acc (|S~_alpha|,
 * int64), each num_nodes long; any may be NULL.                             */
hapod_status hapod_plan_query(hapod_plan_t plan, double* eps, int32_t* level,
                              int64_t* acc);

/* Device memory of a plan's runs, in bytes (host outputs, either may be NULL):
 *   worst_case_bytes     an upper bound on what a run holds at once if every
 *                        node kept all its inputs (rank = input count, at most
 *                        its rows): per level the outputs still alive plus the
 *                        level's outputs and batch scratch.  The ranks of
 *                        Def. 3.2 are data-dependent, so a run usually needs
 *                        far less (a chain's worst case grows with its length).
 *   last_run_peak_bytes  the most the plan's pool held during the last run
 *                        (0 before the first).
 * hapod_plan itself returns HAPOD_E_NOMEM when mem_cap_bytes is below the
 * scratch the leaf level needs whatever the ranks; beyond that the cap is
 * enforced by every allocation of a run (HAPOD_E_NOMEM, the plan stays
 * usable).                                                                  */
hapod_status hapod_plan_workspace(hapod_plan_t plan, int64_t* worst_case_bytes,
                                  int64_t* last_run_peak_bytes);

/* One local POD of node `node` (-1 = root) exactly as a run of the plan
 * computes it (Def. 2.5 with the node's Thm. 3.5 tolerance eps(node), the
 * plan's precision and route: pass-through for eps = 0, the sketched route
 * for nodes of at least 2 sketch_cols inputs, the QR route under qr_pod, else
 * the method of snapshots with the plan's eigensolver choice and tile
 * tuning), on input columns the caller supplies.
 *   S    device, rows(node) x m, ld lds, storage type of the plan (rows(node):
 *        n, or the node's leaf_rows / the most of its children's).
 *   out  device, rows(node) x m capacity, ld ldo: the first *rank columns get
 *        the modes, scaled (sigma_k phi_k) below the root, orthonormal at it.
 *   sigma  host, m capacity.
 * Scratch from the plan's pool.  Synchronises the stream.                  */
hapod_status hapod_plan_node_pod(hapod_plan_t plan, int32_t node, const void* S, int64_t lds,
                                 int64_t m, void* out, int64_t ldo, double* sigma,
                                 int64_t* rank, void* stream);

/* Leaf provider: returns in *ptr a device pointer to the leaf's
 * leaf_rows[leaf] x leaf_cols[leaf] snapshot matrix (column-major, storage
 * type of the plan's precision) and its leading dimension in *ld.  Called
 * once per leaf per run, just before the launch group that first reads it:
 * the leaf's own group, or for a pass-through leaf (eps = 0) its parent's.
 * The data must stay valid until that group has completed; hapod_run
 * synchronises the stream at the end of every group, before the provider
 * is called again, so a provider may stream leaves through a few reused
 * buffers (with leaf_wave bounding how many one group needs).  Non-zero
 * return aborts the run with HAPOD_E_CALLBACK.
 * After a group that read leaves has completed, the provider is called once
 * with leaf = -1 (ptr and ld NULL): no leaf handed over so far is read again,
 * so their memory may be released.  It must return 0 for that call.        */
typedef int32_t (*hapod_leaf_fn)(void* user, int32_t leaf, const void** ptr,
                                 int64_t* ld, void* stream);

/* Run the HAPOD (Def. 3.2) level by level.  All nodes of one level go
 * through one batched sequence of launches (Gram, reduction, eigensolve,
 * truncation, lift); ranks are read back between levels to size the next
 * one.  Intermediate node outputs are released once their parent is done;
 * the root's modes and the per-node ranks and singular values are kept in
 * the plan until the next run or hapod_destroy.  Synchronises the stream.
 * Device memory comes from a pool owned by the plan: blocks a run frees stay
 * cached for the next run (a repeated run maps no new memory), bounded by
 * mem_cap_bytes when set; they are returned to the device when an
 * allocation fails, and by hapod_destroy.
 * Environment: HAPOD_TWIN_BUDGET (bytes) caps the arena that holds the
 * pre-split twins of a level's split-BF16 nodes whose tuned Gram tile is
 * narrower than 128 columns (by default half of the free device memory);
 * HAPOD_GRAM_ITEMS sets the work items a Gram launch aims for (default
 * 8192; row chunks are added until the tile pairs reach it);
 * HAPOD_VERBOSE=1 prints the Krylov eigensolver's progress and the device
 * memory the plan maps and returns to stderr.      */
hapod_status hapod_run(hapod_plan_t plan, hapod_leaf_fn get_leaf, void* user,
                       void* stream);

/* Results of the last run.  node = -1 means the root.
 *   rank   host: |HAPOD(node)|.
 *   sigma  host, rank doubles, may be NULL.
 *   U      device, n x rank, ld ldu, storage type of the plan, may be NULL;
 *          only the root's modes are kept (orthonormal unless the root's
 *          tolerance is 0, in which case they are its input vectors and
 *          sigma is 1).
 * Synchronises the stream.                                                  */
hapod_status hapod_modes(hapod_plan_t plan, int32_t node, void* U, int64_t ldu,
                         double* sigma, int64_t* rank, void* stream);

/* Right factor of the low-rank factorisation of the snapshot map (Rem. 3.8,
 * Def. 3.9): S ~ U diag(sigma) W^T with W^T W = I and the squared Frobenius
 * error at most the sum of eps(gamma)^2 over all nodes.  W is composed from
 * the nodes' right singular vectors, Lambda~ = diag(Lambda~_children)
 * Lambda_node (identity for eps = 0), on the device.
 *   W    device, |S| x N_root double, column-major, ld ldw >= |S|; row i
 *        belongs to snapshot i counted over the leaves in ascending node id,
 *        each leaf's columns in order.
 * Needs a completed run of a plan made with right_vectors = 1
 * (HAPOD_E_INVALID otherwise).  Synchronises the stream.                   */
hapod_status hapod_right_vectors(hapod_plan_t plan, double* W, int64_t ldw, void* stream);

/* The route each node took in the last run.                                */
typedef enum {
  HAPOD_ROUTE_PASSTHROUGH = 0, /* eps = 0: the input vectors, sigma = 1 (Def. 2.5); for the
                                  root (omega = 0) its "modes" are not orthonormal            */
  HAPOD_ROUTE_SNAPSHOTS = 1,   /* the method of snapshots (Gram, eigensolve, truncation, lift) */
  HAPOD_ROUTE_QR = 2,          /* the QR route of hapod_node_pod_qr (plan option qr_pod)      */
  HAPOD_ROUTE_SKETCH = 3,      /* the sketched route of hapod_node_pod_sketch (sketch_cols)   */
  HAPOD_ROUTE_FULL_LEAF = 4    /* a leaf through the method of snapshots up to the truncation,
                                  which kept every column: its own columns went to the parent
                                  (plan option leaf_passthrough); sigma as computed            */
} hapod_route;
/* route: host, one int32 (a hapod_route) for node (-1 = root).
 * HAPOD_E_STATE before the first completed run.                             */
hapod_status hapod_node_route(hapod_plan_t plan, int32_t node, int32_t* route);

/* Diagnostics of a node that took the sketched route in the last run
 * (node = -1: the root).  out13: host, 13 doubles {ell, residual energy r,
 * Cholesky-QR passes on Y, passes on B^T, Jacobi sweeps, then device ms of:
 * sketch Y = S Omega, Q = orth(Y), B = Q^T S, residual, small SVD, modes,
 * then the test matrix of the result (0 sparse sign map, 1 Gaussian), then
 * the columns of the basis in the residual product (ell, or the rank N when
 * the residual was taken against the kept modes; see
 * hapod_node_pod_sketch)}; the counts and times are those of the attempt
 * that gave the result.
 * HAPOD_E_STATE if there is no completed run or the node took another route. */
hapod_status hapod_sketch_stats(hapod_plan_t plan, int32_t node, double* out13);

/* Per-node diagnostics of the last run, host, num_nodes entries each, any may
 * be NULL: input columns m, negative Gram eigenvalues, lambda_1, lambda_min. */
hapod_status hapod_node_stats(hapod_plan_t plan, int64_t* m_in, int64_t* n_negative,
                              double* lambda1, double* lambda_min);

/* Device time in milliseconds of the phases of the last run, measured with
 * HIP events on the run's stream: {total, gram, eig, truncate, lift, reorth}. */
hapod_status hapod_run_timing(hapod_plan_t plan, double* ms6);

/* How the last run's batches of method-of-snapshots nodes (Rem. 2.3; one
 * level, or one wave of leaves) went, host, 3 values:
 *   out3[0]  device-driven batches: every node's eigensolve needs no host
 *            step (Jacobi, or the Householder reduction of 65..256 columns),
 *            so the Gram, eigensolve, truncation (Def. 2.5) and lift run as
 *            one launch sequence with nothing read back in between; outputs
 *            and lift work lists are sized before the ranks are known (for
 *            the node's rank in the previous run, else for m) and the lift's
 *            tiles past the rank retire at once;
 *   out3[1]  batches with the ranks read back before the lift (wide nodes on
 *            Lanczos, right-vector runs, worst-case outputs above a quarter
 *            of the free device memory, or HAPOD_HOST_LEVELS=1);
 *   out3[2]  device-driven batches run again that way because a rank
 *            outgrew the output sized for it (counted here, not in out3[0]). */
hapod_status hapod_plan_batch_stats(hapod_plan_t plan, int64_t* out3);

/* hipGraphs of the last run (option graph_levels), host: out2 = {batches
 * captured, batches replayed}; *graph_ms (may be NULL) the device time of
 * their launches, measured with HIP events on the run's stream.           */
hapod_status hapod_plan_graph_stats(hapod_plan_t plan, int64_t* out2, double* graph_ms);

/* Device time in milliseconds of the phases of one level (1 = leaves) of the
 * last run, measured with HIP events on the run's stream around that level's
 * launches: {gram, eigensolve, truncate, lift}.  ms4: host, 4 doubles.      */
hapod_status hapod_level_timing(hapod_plan_t plan, int32_t level, double* ms4);

void hapod_destroy(hapod_plan_t plan);

const char* hapod_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HAPOD_H */
