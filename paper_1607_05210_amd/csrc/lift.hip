// Batched mode lift out = S B (Rem. 2.3, Def. 3.2): S is n x m (column
// pointers), B the row-major lift operand written by the truncation kernel,
// N (the node's rank) read from device memory; tiles beyond N retire at once.
//
// Work item = (node, 128-row tile, 128-column tile); four wavefronts per
// workgroup, each a 64 x 64 sub-tile of 16 x 16 MFMA blocks.  The MFMA rows
// are snapshot rows (16 consecutive lanes read 16 consecutive doubles of one
// column: coalesced), the reduction index is the snapshot column, and the
// B operand is read along its rows (again 16 consecutive elements).
#include "internal.hpp"
#include "mfma.hpp"

namespace hapod {
namespace {

constexpr int TM = kLiftTileM, TN = kLiftTileN, WT = 64, NB = WT / 16;

template <int C> struct LiftTraits;
template <> struct LiftTraits<0> { using Elem = double; using Acc = d4; static constexpr int KS = 4; };
template <> struct LiftTraits<1> { using Elem = float; using Acc = f4; static constexpr int KS = 4; };
template <> struct LiftTraits<2> { using Elem = float; using Acc = f4; static constexpr int KS = 32; };

template <int C>
__global__ __launch_bounds__(256) void lift_kernel(const LiftNode* __restrict__ nodes, int num_nodes) {
  using Tr = LiftTraits<C>;
  using Elem = typename Tr::Elem;
  using Acc = typename Tr::Acc;
  constexpr int KS = Tr::KS;

  const int item = xcd_item(blockIdx.x, gridDim.x);
  int ni = 0;
  while (ni + 1 < num_nodes && nodes[ni + 1].item_base <= item) ++ni;
  const LiftNode nd = nodes[ni];
  // column tiles of one row stripe are adjacent: they land on the same XCD
  // and share that stripe of S through its L2
  const int local = item - nd.item_base;
  const int rt = local / nd.col_tiles, ct = local % nd.col_tiles;
  const int64_t N = *nd.rank;
  if ((int64_t)ct * TN >= N) return;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int li = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)rt * TM + wi * WT;
  const int64_t n0 = (int64_t)ct * TN + wj * WT;
  if (r0 >= nd.n || n0 >= N) return;

  Acc acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  const int m = nd.m;
  for (int k0 = 0; k0 < m; k0 += KS) {
    if constexpr (C == 0 || C == 1) {
      const int k = k0 + g;
      const Elem* col = (k < m) ? reinterpret_cast<const Elem*>(nd.cols[k]) : nullptr;
      const int64_t rbs = (k < m) ? nd.rbs[k] : kRowBlock;
      const int64_t rows = (k < m) ? nd.crows[k] : 0;
      Elem va[NB];
      double vb[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int64_t row = r0 + a * 16 + li;
        va[a] = (row < rows) ? col[blk_off(row, rbs)] : Elem(0);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int64_t nn = n0 + b * 16 + li;
        vb[b] = (k < m && nn < N) ? nd.B[(int64_t)k * nd.ldb + nn] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if constexpr (C == 0) acc[a][b] = mfma_f64(va[a], vb[b], acc[a][b]);
          else acc[a][b] = mfma_f32(va[a], (float)vb[b], acc[a][b]);
        }
    } else {
      // split-BF16: lane covers reduction slots 8g..8g+7 of this 32-wide step
      float xa[NB][8], xb[NB][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * g + e;
        const float* col = (k < m) ? reinterpret_cast<const float*>(nd.cols[k]) : nullptr;
        const int64_t rbs = (k < m) ? nd.rbs[k] : kRowBlock;
        const int64_t rows = (k < m) ? nd.crows[k] : 0;
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const int64_t row = r0 + a * 16 + li;
          xa[a][e] = (row < rows) ? col[blk_off(row, rbs)] : 0.f;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int64_t nn = n0 + b * 16 + li;
          xb[b][e] = (k < m && nn < N) ? (float)nd.B[(int64_t)k * nd.ldb + nn] : 0.f;
        }
      }
      bf8 ha[NB], la[NB], hb[NB], lb[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) split_bf16x8(xa[a], ha[a], la[a]);
#pragma unroll
      for (int b = 0; b < NB; ++b) split_bf16x8(xb[b], hb[b], lb[b]);
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[a][b] = mfma_bf16(la[a], hb[b], acc[a][b]);
          acc[a][b] = mfma_bf16(ha[a], lb[b], acc[a][b]);
          acc[a][b] = mfma_bf16(ha[a], hb[b], acc[a][b]);
        }
    }
  }

  Elem* out = reinterpret_cast<Elem*>(nd.out);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + a * 16 + acc_row<Acc>(lane, v);
        const int64_t col = n0 + b * 16 + acc_col(lane);
        if (row < nd.n && col < N) out[col * nd.ocs + blk_off(row, nd.obs)] = (Elem)acc[a][b][v];
      }
}

}  // namespace

hapod_status launch_lift(int compute, const LiftNode* d_nodes, int num_nodes, int num_items,
                         hipStream_t stream) {
  if (num_items <= 0) return HAPOD_OK;
  switch (compute) {
    case 0: hipLaunchKernelGGL(lift_kernel<0>, dim3(num_items), dim3(256), 0, stream, d_nodes, num_nodes); break;
    case 1: hipLaunchKernelGGL(lift_kernel<1>, dim3(num_items), dim3(256), 0, stream, d_nodes, num_nodes); break;
    case 2: hipLaunchKernelGGL(lift_kernel<2>, dim3(num_items), dim3(256), 0, stream, d_nodes, num_nodes); break;
    default: set_error("launch_lift: unknown compute mode"); return HAPOD_E_INVALID;
  }
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
