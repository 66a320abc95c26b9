// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hapod.h"

namespace hapod {

// ---- error plumbing --------------------------------------------------------
void set_error(const std::string& msg);

#define HAPOD_HIP(call)                                                       \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::hapod::set_error(std::string(#call) + ": " + hipGetErrorString(e_));  \
      return (e_ == hipErrorOutOfMemory) ? HAPOD_E_NOMEM : HAPOD_E_DEVICE;    \
    }                                                                         \
  } while (0)

#define HAPOD_TRY(expr)                 \
  do {                                  \
    hapod_status s_ = (expr);           \
    if (s_ != HAPOD_OK) return s_;      \
  } while (0)

// ---- storage of a column ---------------------------------------------------
// Rows are grouped in blocks of kRowBlock.  Element r of a column starting at
// p lives at p[(r / kRowBlock) * rbs + r % kRowBlock]: rbs == kRowBlock is a
// plain column-major column; rbs == m_cap * kRowBlock is a column of a
// row-block-tiled n x m_cap buffer (all columns of one 128-row block stored
// contiguously), the layout of every buffer the library owns.
constexpr int kRowBlock = 128;
__host__ __device__ inline int64_t blk_off(int64_t r, int64_t rbs) {
  return (r >> 7) * rbs + (r & (kRowBlock - 1));
}

// ---- batched Gram ----------------------------------------------------------
// One node's input: m columns, column j starting at cols[j] with row-block
// stride rbs[j] (device arrays), rows [0, n).  The upper triangle is cut into
// tile x tile blocks (tile = 128, 64, 32 or 16); rows are split into nchunks
// chunks of chunk_rows.
//   tile 128: the four wavefronts of a workgroup own the four 64 x 64
//             quadrants of the tile.  With nchunks == 1 the tile goes straight
//             into G (both triangles); otherwise into partial slot
//             (pair * nchunks + chunk).
//   tile <= 64: every wavefront computes the whole tile over its own quarter
//             of the chunk's 128-row blocks and writes partial slot
//             (pair * nchunks + chunk) * 4 + wave.
// Partial slots hold tile * tile doubles (column-major) and are summed in
// slot order by gram_reduce.
constexpr int kGramTile = 128;

struct GramNode {
  const void* const* cols;
  const int64_t* rbs;
  const int64_t* crows; // rows held by each column (<= n); rows past it read as 0
  int64_t n;
  int64_t chunk_rows;
  double* G;
  double* partial;
  int64_t ldg;
  int32_t m;
  int32_t nchunks;
  int32_t ntiles;      // ceil(m / tile)
  int32_t pair_base;   // first tile-pair index of this node in the level
  int32_t split;       // 1: columns hold split-BF16 blocks (see launch_split_cols)
  int32_t tile;        // 128, 64, 32 or 16
  // cross > 0: a cross product instead of a Gram matrix.  Columns [0, cross)
  // are the left operand L, columns [cross, m) the right operand Rt; items
  // cover only tile pairs (ti < cross / tile <= tj), numbered compactly
  // (local pair = ti * (ntiles - cross / tile) + tj - cross / tile), and
  // entry (i, j) of L^T Rt goes to G[i * ldg + j] (that is, (L^T Rt)^T
  // column-major with leading dimension ldg, or L^T Rt row-major).
  // cross is a multiple of tile (128-column tiles only).
  int32_t cross;
  int32_t pad;
};
__host__ __device__ inline int gram_slots_per_chunk(int tile) { return tile >= kGramTile ? 1 : 4; }

struct GramItem {
  int32_t node;
  int16_t ti, tj;
  int32_t chunk;
  int32_t pair;        // tile-pair index within the level
  // rows past this are zero in every column of one of the two tiles (each
  // column's rows past its own count read as zero): the item's row range is
  // clipped to it; an item that starts past it writes a zero partial
  int64_t rlim = INT64_MAX;
};

// compute: 0 = FP64 MFMA (double storage), 1 = FP32 MFMA (float storage),
//          2 = split-BF16 x3 (float storage), 3 = FP64 MFMA (float storage)
// Items of one tile size go in one launch: launches[i] covers items
// [first, first + count) of d_items, all of nodes with that tile.  The reduce
// pass covers num_reduce (pair, node) entries over tiles up to max_tile.
// vec: every column of these nodes starts 16-byte aligned and the chunk
// length is a multiple of the MFMA batch, so runs are read as vectors;
// vec = 2: every node is pre-split split-BF16 with 128-column tiles, staged
// through LDS.
// compute >= 0 overrides the launch_gram compute mode for these items.
struct GramLaunch {
  int32_t tile;
  int32_t vec;
  int32_t first;
  int32_t count;
  int32_t compute;
};
// Gram entries set instead of computed (block-structured inner-node Gram):
// rows [r0, r0 + rn) x columns [c0, c0 + cn) of G lie inside one child's
// block diag(sigma^2); entries with row <= col get sigma_row^2 on the
// diagonal and 0 elsewhere, written to both triangles.  s2_base[s2_off + c]
// is sigma_c^2 for the node's column c.
struct GramFill {
  double* G;
  int64_t ldg;
  int64_t s2_off;
  int32_t r0, c0, rn, cn;
};
hapod_status launch_gram_fill(const GramFill* d_fills, int count, const double* s2_base, hipStream_t stream);
// the split-BF16 form computes the Gram of nodes wider than 64 columns with
// split-BF16 products (128-column tiles that split FP32 values into hi / lo
// as they are staged through LDS); narrower nodes, whose tiles are too small
// to pay for the splitting, use FP32 MFMA
constexpr int64_t kBf16MinCols = 65;
// widest split-BF16 node whose 128-column tiles split while staging (two
// column blocks); wider nodes read a pre-split twin (measured on the 2^20 x
// 8192 root: 319 ms from the twin, 638 ms splitting in every tile)
constexpr int64_t kStageSplitMaxCols = 256;
// Gram tile for a node of m columns (16, 32, 64 or 128)
int gram_tile_for(int64_t m);
// row chunks of an n-row node: enough for about target_items work items over
// `pairs` tile pairs, each chunk at least min_rows rows
int pick_chunks(int64_t n, int pairs, int target_items, int64_t min_rows);
hapod_status launch_gram(int compute, const GramNode* d_nodes, const GramItem* d_items,
                         const GramLaunch* launches, int num_launches,
                         const int32_t* d_reduce_pairs, const int32_t* d_reduce_node, int num_reduce,
                         int max_tile, hipStream_t stream);

// ---- batched Jacobi eigensolver -------------------------------------------
struct EigNode {
  double* G;        // m x m, ld = ldg, input (upper triangle read)
  double* work;     // 2 * m2 * m2 doubles (global variant) scratch
  double* Vwork;    // 2 * m * m2 doubles scratch
  double* lambda;   // m outputs (descending)
  double* V;        // m x m outputs, ld = ldv
  int64_t ldg;
  int64_t ldv;
  int32_t m;
  int32_t pad;
  int32_t* sweeps;  // 1 int output (may be null)
};
constexpr int kJacobiLdsMax = 128;   // packed double-buffered upper triangle fits in LDS
constexpr int kJacobiMax = 1024;     // global-memory variant limit
hapod_status launch_jacobi(const EigNode* d_nodes, int num_nodes, int max_m,
                           hipStream_t stream);
size_t jacobi_work_doubles(int m);
size_t jacobi_vwork_doubles(int m);

// ---- batched truncation ----------------------------------------------------
// policy: 0 = clamp negatives (Def. 2.5 on the computed spectrum),
//         1 = clip the rounding band |lambda| <= theta,
//             theta = max(-lambda_min, floor_abs)
struct TruncNode {
  const double* lambda;   // m, descending
  const double* V;        // m x m, ld ldv (eigenvectors)
  double* B;              // lift operand, row-major m x ldb
  float* B32;             // the same in FP32 (may be null): the FP32 and
                          // split-BF16 lifts read this one
  double* sigma;          // m outputs (first N valid)
  int64_t* rank;          // 1 output
  double* info;           // 6 outputs: tail(N), lambda1, lambda_min, n_neg, theta, rank_clamp
  double eps2;
  double floor_abs;
  int64_t ldv;
  int64_t ldb;
  int32_t m;
  int32_t policy;
  int32_t root;           // 1: B = V Lambda^{-1/2}, else B = V
  int32_t pad;
  const double* floor_ptr;  // non-null: floor_abs is read from here (written
                            // on the device by the eigensolve)
};
hapod_status launch_truncate(const TruncNode* d_nodes, int num_nodes, hipStream_t stream);
// B[k * ldb + n] = V[k][n] (lambda == nullptr) or V[k][n] / sqrt(lambda[n]);
// B32 (may be null) gets the same values rounded to FP32
hapod_status launch_lift_operand(const double* V, int64_t ldv, const double* lambda, int64_t m, int64_t N,
                                 double* B, float* B32, int64_t ldb, hipStream_t stream);
// dst[i] = (float)src[i], i < count
hapod_status launch_to_f32(const double* src, float* dst, int64_t count, hipStream_t stream);

// ---- batched lift -----------------------------------------------------------
// out = S * B[:, :N] where S is given by column pointers (m columns, n rows)
// and B is row-major (ldb), N read from *rank on the device.
constexpr int kLiftTileM = 128;
constexpr int kLiftTileN = 128;
struct LiftNode {
  const void* const* cols;
  const int64_t* rbs;
  const int64_t* crows;  // rows held by each column; rows past it read as 0
  const double* B;       // FP64 lift (compute 0): row-major, ldb
  const float* B32;      // FP32 and split-BF16 lifts: the same operand in FP32
  const int64_t* rank;   // device pointer to N
  void* out;             // element (r, c) at out[c * ocs + blk_off(r, obs)]
  int64_t n;
  int64_t ldb;
  int64_t ocs;           // column stride: ld (plain) or kRowBlock (tiled)
  int64_t obs;           // row-block stride: kRowBlock (plain) or m_cap * kRowBlock
  int32_t m;
  int32_t row_tiles;
  int32_t col_tiles;     // worst case ceil(maxN / TN)
  int32_t item_base;
  int32_t rt_per;        // row tiles per work item (0 or 1: one); the node's
                         // items are ceil(row_tiles / rt_per) x col_tiles
  int32_t pad;
  // Residual mode (launch_lift_residual, FP64 only): instead of storing the
  // product P = S B, every output column c is compared with column c of a
  // second matrix T (column table rcols / rrbs / rrows, N columns, n rows):
  // the sum over the work item's rows of (T - P)^2 goes to
  // rpart[(row_group * 2 + h) * N + c], h the half (64 rows) of each
  // 128-row tile.  Row groups are the items' ceil(row_tiles / rt_per).
  const void* const* rcols;
  const int64_t* rrbs;
  const int64_t* rrows;
  double* rpart;
  // Split-BF16 lift (compute 2): the lift operand split once into BF16 hi
  // and lo, transposed: for output column c < N and reduction stage s
  // (reduction indices 32 s .. 32 s + 31, zero past m), 128 bytes at
  // Bs + (c * ceil(m / 32) + s) * 128, the 32 hi then the 32 lo values.
  // Written from B32 by launch_split_operand; room for m columns (N <= m).
  char* Bs;
  // > 0: the output holds only this many columns; columns past it are not
  // written (a device-driven batch sized the output before the rank was
  // known and checks the rank afterwards)
  int64_t ncap;
};
// compute: 0 FP64 MFMA, 1 FP32 MFMA, 2 split-BF16 (three BF16 products per
// term on BF16 MFMA, FP32 accumulation; reads Bs); output storage = input
// storage.
// narrow: every node has N <= 64 and its tiles are kLiftNarrowM x 64
// (row_tiles and col_tiles counted for that tile).
constexpr int kLiftNarrowM = 256;
hapod_status launch_lift(int compute, const LiftNode* d_nodes, int num_nodes,
                         int num_items, hipStream_t stream, bool narrow = false);
// Bs of every node from its B32, the first *rank columns (max_m: the widest
// node's m, for the grid)
hapod_status launch_split_operand(const LiftNode* d_nodes, int num_nodes, int64_t max_m, hipStream_t stream);
inline size_t split_operand_bytes(int64_t m) { return (size_t)((m + 31) / 32) * 128 * (size_t)m; }
// Residual mode of the FP64 lift (see LiftNode::rcols), one node.
// dense: every column of the node holds all n rows, may be read to the next
// multiple of 128 rows, every column and row block starts 16-byte aligned,
// m is a multiple of 8, and the operand B starts 16-byte aligned with ldb a
// multiple of 4 (or N a multiple of 128 and ldb even): the operand loads then
// carry no guards.
hapod_status launch_lift_residual(const LiftNode* d_node, int num_items, hipStream_t stream, bool dense = false);
// The FP64 lift (128 x 128 tiles) of nodes that all meet the dense conditions
// above.
hapod_status launch_lift_dense(const LiftNode* d_nodes, int num_nodes, int num_items, hipStream_t stream);
// res[c] = sum over g < groups of rpart[g * N + c], in order of g
hapod_status launch_sum_partials(const double* rpart, int64_t groups, int64_t N, double* res, hipStream_t stream);

// ---- helpers ----------------------------------------------------------------
hapod_status launch_fill_colptrs(const void* base, int64_t ld, int64_t m, int elem_bytes,
                                 const void** d_out, hipStream_t stream);
hapod_status launch_copy_cols(int elem_bytes, int64_t n, int64_t m, const void* const* cols,
                              const int64_t* rbs, const int64_t* crows, void* out, int64_t ldo,
                              hipStream_t stream);
hapod_status launch_zero_bytes(void* p, size_t bytes, hipStream_t stream);
// C = A B (column-major FP64, M x K times K x N; ld >= rows)
hapod_status launch_dgemm_nn(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                             int64_t ldb, double* C, int64_t ldc, hipStream_t stream);
// T = I (n x n, ld ld)
hapod_status launch_set_identity(double* T, int64_t n, int64_t ld, hipStream_t stream);
hapod_status launch_check_diag(const double* G, int64_t ldg, int64_t m, int32_t* d_flag,
                               hipStream_t stream);
hapod_status launch_set_scalar_i64(int64_t* p, int64_t v, hipStream_t stream);
hapod_status launch_fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t stream);
// Split-BF16 twin of m float columns (pointer + row-block stride each) into a
// row-block-tiled buffer of capacity m: block b of column c occupies the 128
// float slots at dst + (b * m + c) * 128 and holds 128 bf16 hi values followed
// by 128 bf16 lo values (x = hi + lo + O(2^-17 |x|)); rows past n are zero.
hapod_status launch_split_cols(int64_t n, int64_t m, const void* const* cols, const int64_t* rbs,
                               const int64_t* crows, float* dst, hipStream_t stream);

// ---- Cholesky-QR re-orthonormalisation -------------------------------------
hapod_status launch_chol_inv(double* W, int64_t ldw, int64_t N, double* Rinv, int64_t ldr,
                             int32_t* d_bad, hipStream_t stream, double rel_floor = 1e-12);

// ---- accuracy-preserving local POD (qr.hip) -------------------------------------
constexpr int64_t kQrMaxM = 512;     // widest node of the QR-based POD
constexpr int64_t kOsjLdsMaxM = 128; // the Jacobi SVD keeps R in LDS up to this width
constexpr int kQrMaxPasses = 12;     // Cholesky-QR passes before giving up
constexpr int kCholLdsMaxN = 128;    // launch_chol_inv keeps both triangles in LDS up to this N
constexpr int kCholWgMaxN = 1024;    // and works in place in global memory up to this N
hapod_status launch_chol_inv_wg(double* W, int64_t ldw, int64_t N, double* Rinv, int64_t ldr, int32_t* d_bad,
                                hipStream_t stream, double rel_floor);
// G[k][k] += coef * trace(G)
hapod_status launch_shift_diag(double* G, int64_t ldg, int64_t m, double coef, hipStream_t stream);
// dst (n x m) = the columns of a column table (device arrays), rows past a
// column's row count zero; dst plain (ld n) for dst_rbs == 0, else
// row-block-tiled with that row-block stride
hapod_status launch_gather_cols(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n,
                                int64_t m, double* dst, int64_t dst_rbs, hipStream_t stream);
// out[0] = max over the upper triangle of |G_ij - delta_ij|
hapod_status launch_identity_dev(const double* G, int64_t ldg, int64_t m, double* out, hipStream_t stream);
// zero[j] |= (G_jj == 0); with D (non-null): D_j = sqrt(G_jj) (1 for zero
// columns) and G <- D^-1 G D^-1; zero columns' diagonal set to 1
hapod_status launch_gram_zero_scale(double* G, int64_t ldg, int64_t m, int32_t* zero, double* D, hipStream_t stream);
// R (column-major) column j *= D_j, Rinv (row-major) row i /= D_i
hapod_status launch_unscale_factors(double* R, int64_t ldr, double* Rinv, int64_t ldi, int64_t m, const double* D,
                                    hipStream_t stream);
// row j of R (column-major) = 0 where zero[j]
hapod_status launch_zero_rows(double* R, int64_t ldr, int64_t m, const int32_t* zero, hipStream_t stream);
// R = upper triangle of W, zeros below (both column-major)
hapod_status launch_triu(const double* W, int64_t ldw, int64_t N, double* R, int64_t ldr, hipStream_t stream);
// one-sided Jacobi SVD of A (m x m, column-major, ld m, overwritten): sigma
// (device, m, descending), B (device, row-major m x m): column p is the
// p-th left singular vector times sigma_p (scaled) or alone; info (device, 2
// int32): info[0] = sweeps taken or -1 without convergence, info[1] scratch.
// m <= 64: one workgroup with A in LDS (asynchronous); above, block Jacobi
// over blocks of 16 columns, one launch per round and a readback per sweep
// (synchronises the stream).
hapod_status launch_osj(double* A, int64_t m, double* sigma, double* B, int scaled, int32_t* info,
                        hipStream_t stream);

// ---- sketched local POD (sketch.hip) -----------------------------------------
// out[i] ~ N(0, 1), i < count, from a counter-based generator (deterministic
// for a seed, independent of the launch shape)
hapod_status launch_normal_fill(double* out, int64_t count, uint64_t seed, hipStream_t stream);
// T = A^T for a square m x m matrix (both column-major)
hapod_status launch_transpose(const double* A, int64_t lda, int64_t m, double* T, int64_t ldt, hipStream_t stream);
// C (row-major, ld ld, rows_c + cols rows): the first rows_c rows negated,
// the next cols rows the identity
hapod_status launch_neg_ident(double* C, int64_t rows_c, int64_t cols, int64_t ld, hipStream_t stream);
// R[(c0 + j) * ldr + i] += C[i * ldc + j] for i < rows, j < cols: a row-major
// block added, transposed, into column-major R
hapod_status launch_acc_transposed(double* R, int64_t ldr, int64_t c0, const double* C, int64_t ldc, int64_t rows,
                                   int64_t cols, hipStream_t stream);
constexpr int64_t kSketchMaxCols = 512;  // widest sketch (the Jacobi SVD's limit)
constexpr int kSignNnz = 8;              // nonzeros per row of the sparse sign map
constexpr int kSketchRows = 64;          // rows of S per workgroup of the sparse sketch
constexpr int kSketchDepth = 2;          // column chunks the sparse sketch loads ahead
// Y = S Omega for the sparse sign map of (m, ell, seed) in its block-shifted
// form (entries +-1/sqrt(kSignNnz); ell = 128, 256, 384 or 512): S an n-row
// column table of m columns (device arrays; full_rows: rows every column
// holds; 8-byte alignment), Y element (r, c) at Y[c * ocs + blk_off(r,
// obs)], rows < n written.
hapod_status launch_sign_sketch(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n,
                                int64_t m, int64_t full_rows, uint64_t seed, int64_t ell, double* Y, int64_t ocs,
                                int64_t obs, hipStream_t stream);

}  // namespace hapod
