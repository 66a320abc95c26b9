// Batched mode lift out = S B (Rem. 2.3, Def. 3.2): S is n x m (column
// pointers), B the row-major lift operand written by the truncation kernel,
// N (the node's rank) read from device memory; tiles beyond N retire at once.
//
// Work item = (node, 128-row tile, 128-column tile); four wavefronts per
// workgroup, each a 64 x 64 sub-tile held as 4 x 4 blocks of 16 x 16 MFMA
// accumulators.  The MFMA row index is the snapshot row and the reduction
// index the snapshot column.  Rows and output columns are permuted inside the
// wavefront's sub-tile so that each lane reads contiguous runs: MFMA row i of
// block a is sub-tile row 4 i + a (lane i loads rows 4 i .. 4 i + 3 of one
// column in one vector load), and MFMA column j of block b is sub-tile column
// 4 j + b (a run of 4 consecutive entries of a row of B).  The store undoes
// both permutations.
//
// The column table (pointer, row-block stride, rows held) of the next 1024
// reduction indices is staged in LDS, so the data loads never wait on a
// pointer load; data loads are double-buffered in registers: one batch of
// reduction steps is fetched while the previous one runs on the matrix cores.
#include "internal.hpp"
#include "mfma.hpp"

namespace hapod {
namespace {

constexpr int TM = kLiftTileM, TN = kLiftTileN, WT = 64, NB = WT / 16;
constexpr int KT = 1024;  // reduction indices per LDS column-table chunk (4 per thread)

template <int C> struct LiftTraits;
template <> struct LiftTraits<0> { using Elem = double; using Acc = d4; };
template <> struct LiftTraits<1> { using Elem = float; using Acc = f4; };

// out[t] = p[t] for t < avail (at most 4), else 0; one vector load when the
// run is whole and 16-byte aligned.
__device__ __forceinline__ void run4(const double* p, int64_t avail, double (&out)[4]) {
  if (avail >= 4 && (((uintptr_t)p & 15u) == 0)) {
    const dv2 x = *(gptr<dv2>)as_global(p);
    const dv2 y = *(gptr<dv2>)as_global(p + 2);
    out[0] = x[0]; out[1] = x[1]; out[2] = y[0]; out[3] = y[1];
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = (t < avail) ? p[t] : 0.0;
  }
}
__device__ __forceinline__ void run4(const float* p, int64_t avail, float (&out)[4]) {
  if (avail >= 4 && (((uintptr_t)p & 15u) == 0)) {
    const fv4 x = *(gptr<fv4>)as_global(p);
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = (t < avail) ? p[t] : 0.f;
  }
}

// NARROW (ranks up to 64): a 256 x 64 tile, the four wavefronts stacked
// along the rows, so that no wavefront idles on columns past N.
// RES: the residual mode (LiftNode::rcols): the product is compared with the
// node's second matrix instead of being stored.
// DENSE: every column holds all n rows and may be read to the next multiple
// of 128 rows (row-block-tiled, or n a multiple of 128), every column and
// every row block starts 16-byte aligned, m is a multiple of 8, and the lift
// operand's rows are whole aligned runs (ldb a multiple of 4, or N a multiple
// of 128 with ldb even): operand runs are loaded without guards or branches
// (rows past n and columns past N only reach outputs that are never stored
// or summed).
template <int C, bool NARROW, bool RES = false, bool DENSE = false>
__global__ __launch_bounds__(256, (C == 0) ? 2 : 1) void lift_kernel(const LiftNode* __restrict__ nodes, int num_nodes) {
  static_assert(!RES || (C == 0 && !NARROW), "residual mode: FP64 128 x 128 tiles");
  static_assert(!DENSE || (C == 0 && !NARROW), "dense mode: FP64 128 x 128 tiles");
  constexpr int TMk = NARROW ? 4 * WT : TM;
  constexpr int TNk = NARROW ? WT : TN;
  using Tr = LiftTraits<C>;
  using Elem = typename Tr::Elem;
  using Acc = typename Tr::Acc;
  using BElem = Elem;  // the lift operand comes in the storage precision

  const int item = xcd_item(blockIdx.x, gridDim.x);
  // the node whose item range holds this item: last item_base <= item
  int lo = 0, hi = num_nodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].item_base <= item) lo = mid;
    else hi = mid - 1;
  }
  const LiftNode nd = nodes[lo];
  // column tiles of one row stripe are adjacent: they land on the same XCD
  // and share that stripe of S through its L2
  const int local = item - nd.item_base;
  const int rg = local / nd.col_tiles, ct = local % nd.col_tiles;
  const int64_t N = (nd.ncap > 0) ? min(*nd.rank, nd.ncap) : *nd.rank;
  if ((int64_t)ct * TNk >= N) return;  // whole workgroup
  const int rt_per = max(nd.rt_per, 1);
  const int rt_begin = rg * rt_per, rt_end = min(rt_begin + rt_per, nd.row_tiles);
  // residual mode: per output column of the lane (b), the squared differences
  // over every row the lane sees, in a fixed order
  double ssq[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) ssq[b] = 0.0;

  __shared__ const char* tcol[KT];
  __shared__ int64_t trbs[KT];
  __shared__ int64_t trows[KT];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = NARROW ? wave : (wave >> 1), wj = NARROW ? 0 : (wave & 1);
  const int li = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)ct * TNk + wj * WT;
  const int64_t nl = n0 + 4 * li;   // first of the lane's 4 output columns
  const int64_t bavail = N - nl;
  const BElem* bop;
  if constexpr (C == 0) bop = nd.B;
  else bop = nd.B32;
  const int m = nd.m;
  auto load_table = [&](int kc) {
    for (int t = threadIdx.x; t < KT; t += blockDim.x) {
      const int k = kc + t;
      const bool kv = k < m;
      tcol[t] = kv ? reinterpret_cast<const char*>(nd.cols[k]) : nullptr;
      trbs[t] = kv ? nd.rbs[k] : kRowBlock;
      trows[t] = kv ? nd.crows[k] : 0;
    }
  };
  // with at most KT reduction indices the table is loaded once for all tiles
  const bool one_chunk = (m <= KT);
  if (one_chunk) {
    load_table(0);
    __syncthreads();
  }

  for (int rt = rt_begin; rt < rt_end; ++rt) {
  const int64_t r0 = (int64_t)rt * TMk + wi * WT;
  const bool active = (r0 < nd.n) && (n0 < N);
  const int64_t rl = r0 + 4 * li;   // first of the lane's 4 rows (one row block)
  const int64_t roff = rl & (kRowBlock - 1), rblk = rl >> 7;

  Acc acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  for (int kc = 0; kc < m; kc += KT) {
    if (!one_chunk) {
      __syncthreads();  // the previous chunk's table is no longer read
      load_table(kc);
      __syncthreads();
    }
    if (!active) continue;
    const int kend = min(m, kc + KT);
    // a lane's run of column k (table slot t): up to 4 rows from row rl
    auto srun = [&](int t, Elem (&x)[4]) {
      if constexpr (DENSE) {
        const Elem* p = reinterpret_cast<const Elem*>(tcol[t]) + rblk * trbs[t] + roff;
        const dv2 u = *(gptr<dv2>)as_global(p);
        const dv2 v = *(gptr<dv2>)as_global(p + 2);
        x[0] = u[0]; x[1] = u[1]; x[2] = v[0]; x[3] = v[1];
        return;
      }
      const int64_t avail = trows[t] - rl;
      if (avail <= 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = Elem(0);
      } else {
        run4(reinterpret_cast<const Elem*>(tcol[t]) + rblk * trbs[t] + roff, avail, x);
      }
    };
    auto brun = [&](int k, BElem (&y)[4]) {
      if constexpr (DENSE) {
        // runs past the operand's row (columns >= N, never stored) read
        // the row's last run instead
        const BElem* p = bop + (int64_t)k * nd.ldb + min(nl, nd.ldb - 4);
        const dv2 u = *(gptr<dv2>)as_global(p);
        const dv2 v = *(gptr<dv2>)as_global(p + 2);
        y[0] = u[0]; y[1] = u[1]; y[2] = v[0]; y[3] = v[1];
        return;
      }
      if (k < kend && bavail > 0) run4(bop + (int64_t)k * nd.ldb + nl, bavail, y);
      else {
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = BElem(0);
      }
    };
    // batches of U MFMA steps of 4 reduction indices each
    constexpr int U = (C == 0) ? 1 : 4, KB = 4 * U;
    Elem xa[2][U][4];
    BElem xb[2][U][4];
    auto load = [&](int kb, Elem (&va)[U][4], BElem (&vb)[U][4]) {
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const int k = kb + 4 * t + g;
        if (DENSE || k < kend) srun(k - kc, va[t]);
        else {
#pragma unroll
          for (int a = 0; a < 4; ++a) va[t][a] = Elem(0);
        }
        brun(k, vb[t]);
      }
    };
    auto compute = [&](Elem (&va)[U][4], BElem (&vb)[U][4]) {
#pragma unroll
      for (int t = 0; t < U; ++t)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if constexpr (C == 0) acc[a][b] = mfma_f64(va[t][a], vb[t][b], acc[a][b]);
            else acc[a][b] = mfma_f32(va[t][a], vb[t][b], acc[a][b]);
          }
    };
    load(kc, xa[0], xb[0]);
    for (int kb = kc; kb < kend; kb += 2 * KB) {
      load(kb + KB, xa[1], xb[1]);
      compute(xa[0], xb[0]);
      // dense: the refill is unconditional (the last one re-reads the chunk's
      // last batch, unused), so each wait is for a fixed count of loads and
      // the refill stays in flight under the next batch's products
      if constexpr (DENSE) load(min(kb + 2 * KB, kend - KB), xa[0], xb[0]);
      else if (kb + 2 * KB < kend) load(kb + 2 * KB, xa[0], xb[0]);
      compute(xa[1], xb[1]);
    }
  }
  if (!active) continue;

  if constexpr (RES) {
    // T - P over the lane's rows r0 + 4 acc_row + a of its columns
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t col = n0 + 4 * acc_col(lane) + b;
      if (col >= N) continue;
      const double* tc = reinterpret_cast<const double*>(nd.rcols[col]);
      const int64_t trb = nd.rrbs[col];
      const int64_t tr = min(nd.rrows[col], nd.n);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 4 * acc_row<Acc>(lane, v);
        if (row >= nd.n) continue;
        double t4[4];
        if (row < tr) run4(tc + blk_off(row, trb), tr - row, t4);
        else {
#pragma unroll
          for (int a = 0; a < 4; ++a) t4[a] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double d = (row + a < nd.n) ? t4[a] - (double)acc[a][b][v] : 0.0;
          ssq[b] += d * d;
        }
      }
      // one column block's reads at a time: hoisting all sixteen runs of T
      // above the products would take 128 more registers
      __builtin_amdgcn_sched_barrier(0);
    }
    continue;
  }

  // lane (g, j) holds, for output column n0 + 4 j + b and accumulator
  // register v, the rows r0 + 4 acc_row + a (a = 0..3): four consecutive
  // rows, written as one vector store
  Elem* out = reinterpret_cast<Elem*>(nd.out);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t col = n0 + 4 * acc_col(lane) + b;
    if (col >= N) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * acc_row<Acc>(lane, v);
      Elem* p = out + col * nd.ocs + blk_off(row, nd.obs);
      Elem x[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = (Elem)acc[a][b][v];
      if (row + 4 <= nd.n && (((uintptr_t)p & 15u) == 0)) {
        if constexpr (C == 0) {
          __attribute__((address_space(1))) dv2* q = (__attribute__((address_space(1))) dv2*)p;
          q[0] = dv2{x[0], x[1]};
          q[1] = dv2{x[2], x[3]};
        } else {
          *(__attribute__((address_space(1))) fv4*)p = fv4{x[0], x[1], x[2], x[3]};
        }
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
          if (row + a < nd.n) p[a] = x[a];
      }
    }
  }
  }  // row tiles
  if constexpr (RES) {
    // the four lanes of a column (lane / 16 = 0..3) hold its rows in four
    // interleaved sets: sum them, then one write per (row half, column)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double x = ssq[b];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      const int64_t col = n0 + 4 * acc_col(lane) + b;
      if (g == 0 && col < N) nd.rpart[((int64_t)rg * 2 + wi) * N + col] = x;
    }
  }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ rpart, int64_t groups, int64_t N,
                                                           double* __restrict__ res) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double s = 0.0;
  for (int64_t g = 0; g < groups; ++g) s += rpart[g * N + c];
  res[c] = s;
}

// FP32 tiles with both operands staged through LDS: per stage KS reduction
// indices, the workgroup's 256 threads load the S block (TM rows x KS
// columns) and the B block (KS rows x TN output columns) in 16-byte chunks,
// double-buffered, two workgroups per CU; every lane then reads its 4-row S
// run and 4-column B run from LDS.  Regular tiles are 128 x 128 (KS = 32),
// narrow ones 256 x 64 with the wavefronts stacked along the rows (KS = 16).  The MFMA sequence
// (reduction indices k0 + 4 t + g in step t, blocks a x b) is the one of
// lift_kernel, so the results are identical.  (Measured: 1.4x faster than
// lift_kernel for FP32; the FP64 instance, one workgroup per CU by its
// registers, was 1.4x slower, so FP64 keeps lift_kernel.)
template <int C, bool NARROW>
__global__ __launch_bounds__(256, 2) void lift_staged_kernel(const LiftNode* __restrict__ nodes, int num_nodes) {
  using Tr = LiftTraits<C>;
  using Elem = typename Tr::Elem;
  using Acc = typename Tr::Acc;
  constexpr int EB = (int)sizeof(Elem);
  static_assert(C == 1, "FP32 only");
  constexpr int TMk = NARROW ? 4 * WT : TM;  // tile rows
  constexpr int TNk = NARROW ? WT : TN;      // tile columns
  constexpr int KS = NARROW ? 16 : 32;       // reduction indices per stage
  constexpr int EPC = 16 / EB;               // elements per 16-byte chunk
  constexpr int CPC = TMk * EB / 16;         // chunks per S column
  constexpr int CPR = TNk * EB / 16;         // chunks per B row
  constexpr int SB = TMk * EB + 16;          // LDS bytes per S column (padded)
  constexpr int BBy = TNk * EB + 16;         // LDS bytes per B row (padded)
  constexpr int KTS = 256;                   // column-table chunk
  constexpr int NLS = KS * CPC / 256;        // S chunks per thread and stage
  constexpr int NLB = KS * CPR / 256;        // B chunks per thread and stage
  static_assert(NLS * 256 == KS * CPC && NLB * 256 == KS * CPR && NLB >= 1, "whole chunks per thread");
  typedef __attribute__((ext_vector_type(4))) int i4;

  const int item = xcd_item(blockIdx.x, gridDim.x);
  int lo = 0, hi = num_nodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].item_base <= item) lo = mid;
    else hi = mid - 1;
  }
  const LiftNode nd = nodes[lo];
  const int local = item - nd.item_base;
  const int rg = local / nd.col_tiles, ct = local % nd.col_tiles;
  const int64_t N = (nd.ncap > 0) ? min(*nd.rank, nd.ncap) : *nd.rank;
  if ((int64_t)ct * TNk >= N) return;  // whole workgroup
  const int rt_per = max(nd.rt_per, 1);
  const int rt_begin = rg * rt_per, rt_end = min(rt_begin + rt_per, nd.row_tiles);
  // residual mode: per output column of the lane (b), the squared differences
  // over every row the lane sees, in a fixed order
  double ssq[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) ssq[b] = 0.0;

  __shared__ __attribute__((aligned(16))) char sS[2][KS * SB];
  __shared__ __attribute__((aligned(16))) char sB[2][KS * BBy];
  __shared__ const char* tcol[KTS];
  __shared__ int64_t trbs[KTS];
  __shared__ int64_t trows[KTS];

  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int wi = NARROW ? wave : (wave >> 1), wj = NARROW ? 0 : (wave & 1);
  const int li = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)ct * TNk + wj * WT;
  const Elem* bop;
  if constexpr (C == 0) bop = nd.B;
  else bop = nd.B32;
  const int m = nd.m;
  const int stages = (m + KS - 1) / KS;
  // the table chunk holding stage st (refilled between stages)
  int table_base = -KTS;
  auto ensure_table = [&](int kfirst) {
    if (kfirst >= table_base && kfirst + KS <= table_base + KTS) return;
    __syncthreads();
    table_base = kfirst;
    const int k = kfirst + t;
    const bool kv = k < m;
    tcol[t] = kv ? reinterpret_cast<const char*>(nd.cols[k]) : nullptr;
    trbs[t] = kv ? nd.rbs[k] : kRowBlock;
    trows[t] = kv ? nd.crows[k] : 0;
    __syncthreads();
  };

  for (int rt = rt_begin; rt < rt_end; ++rt) {
    const int64_t rtile = (int64_t)rt * TMk;
    const bool active = (rtile + wi * WT < nd.n) && (n0 < N);
    Acc acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};
    i4 ps0[NLS], pb0[NLB], ps1[NLS], pb1[NLB];  // two stages in flight
    // chunk q = i * 256 + t: S column q / CPC, rows of part q % CPC; B row
    // q / CPR, columns of part q % CPR
    auto gload = [&](int st, i4 (&ps)[NLS], i4 (&pb)[NLB]) {
      const int kfirst = st * KS;
#pragma unroll
      for (int i = 0; i < NLS; ++i) {
        const int q = i * 256 + t;
        const int kk = q / CPC, part = q % CPC;
        const int k = kfirst + kk;
        const int tk = k - table_base;
        const int64_t row = rtile + part * EPC;
        Elem x[EPC];
        const int64_t avail = (k < m) ? trows[tk] - row : 0;
        const char* p = (k < m) ? tcol[tk] + ((row >> 7) * trbs[tk] + (row & (kRowBlock - 1))) * EB : nullptr;
        if (avail >= EPC && (((uintptr_t)p & 15u) == 0)) {
          ps[i] = *(gptr<i4>)as_global(reinterpret_cast<const i4*>(p));
        } else {
#pragma unroll
          for (int e = 0; e < EPC; ++e) x[e] = (e < avail) ? reinterpret_cast<const Elem*>(p)[e] : Elem(0);
          ps[i] = *reinterpret_cast<const i4*>(x);
        }
      }
#pragma unroll
      for (int i = 0; i < NLB; ++i) {
        const int q = i * 256 + t;
        const int kk = q / CPR, part = q % CPR;
        const int k = kfirst + kk;
        const int64_t col = (int64_t)ct * TNk + part * EPC;
        const int64_t avail = (k < m) ? N - col : 0;
        const Elem* p = bop + (int64_t)k * nd.ldb + col;
        Elem x[EPC];
        if (avail >= EPC && (((uintptr_t)p & 15u) == 0)) {
          pb[i] = *(gptr<i4>)as_global(reinterpret_cast<const i4*>(p));
        } else {
#pragma unroll
          for (int e = 0; e < EPC; ++e) x[e] = (e < avail) ? p[e] : Elem(0);
          pb[i] = *reinterpret_cast<const i4*>(x);
        }
      }
    };
    auto lstore = [&](int buf, const i4 (&ps)[NLS], const i4 (&pb)[NLB]) {
#pragma unroll
      for (int i = 0; i < NLS; ++i) {
        const int q = i * 256 + t;
        *(i4*)(sS[buf] + (q / CPC) * SB + (q % CPC) * 16) = ps[i];
      }
#pragma unroll
      for (int i = 0; i < NLB; ++i) {
        const int q = i * 256 + t;
        *(i4*)(sB[buf] + (q / CPR) * BBy + (q % CPR) * 16) = pb[i];
      }
    };
    auto compute = [&](int buf) {
#pragma unroll
      for (int s4 = 0; s4 < KS / 4; ++s4) {
        const int kk = 4 * s4 + g;
        const Elem* sr = reinterpret_cast<const Elem*>(sS[buf] + kk * SB) + wi * WT + 4 * li;
        const Elem* br = reinterpret_cast<const Elem*>(sB[buf] + kk * BBy) + wj * WT + 4 * li;
        Elem va[4], vb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          va[e] = sr[e];
          vb[e] = br[e];
        }
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if constexpr (C == 0) acc[a][b] = mfma_f64(va[a], vb[b], acc[a][b]);
            else acc[a][b] = mfma_f32(va[a], vb[b], acc[a][b]);
          }
      }
    };
    if constexpr (!NARROW) {
      // one stage in flight (a second set of registers would spill here)
      if (stages > 0) {
        ensure_table(0);
        gload(0, ps0, pb0);
        lstore(0, ps0, pb0);
      }
      __syncthreads();
      for (int st = 0; st < stages; ++st) {
        const bool more = st + 1 < stages;
        if (more) {
          ensure_table((st + 1) * KS);
          gload(st + 1, ps0, pb0);
        }
        if (active) compute(st & 1);
        if (more) lstore((st + 1) & 1, ps0, pb0);
        __syncthreads();
      }
    } else {
    // stage s sits in LDS buffer s & 1; the loads of stage s + 2 are issued
    // before stage s is computed, so two stages are in flight (the loop is
    // unrolled by two to keep the register sets static)
    if (stages > 0) {
      ensure_table(0);
      gload(0, ps0, pb0);
      lstore(0, ps0, pb0);
    }
    if (stages > 1) {
      ensure_table(KS);
      gload(1, ps1, pb1);
    }
    __syncthreads();
    for (int st = 0; st < stages; st += 2) {
      if (st + 2 < stages) {
        ensure_table((st + 2) * KS);
        gload(st + 2, ps0, pb0);
      }
      if (active) compute(0);
      if (st + 1 < stages) lstore(1, ps1, pb1);
      __syncthreads();
      if (st + 1 >= stages) break;
      if (st + 3 < stages) {
        ensure_table((st + 3) * KS);
        gload(st + 3, ps1, pb1);
      }
      if (active) compute(1);
      if (st + 2 < stages) lstore(0, ps0, pb0);
      __syncthreads();
    }
    }
    if (!active) continue;
    Elem* out = reinterpret_cast<Elem*>(nd.out);
    const int64_t r0 = rtile + wi * WT;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t col = n0 + 4 * acc_col(lane) + b;
      if (col >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 4 * acc_row<Acc>(lane, v);
        Elem* p = out + col * nd.ocs + blk_off(row, nd.obs);
        Elem x[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = (Elem)acc[a][b][v];
        if (row + 4 <= nd.n && (((uintptr_t)p & 15u) == 0)) {
          if constexpr (C == 0) {
            __attribute__((address_space(1))) dv2* q = (__attribute__((address_space(1))) dv2*)p;
            q[0] = dv2{x[0], x[1]};
            q[1] = dv2{x[2], x[3]};
          } else {
            *(__attribute__((address_space(1))) fv4*)p = fv4{x[0], x[1], x[2], x[3]};
          }
        } else {
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (row + a < nd.n) p[a] = x[a];
        }
      }
    }
  }  // row tiles
}

// Split-BF16 lift: out = S B with every product x y taken as
// xl yh + xh yl + xh yh (x = xh + xl, y = yh + yl, BF16 parts; FP32
// accumulation), on BF16 MFMA (16 x 16 x 32).  Per stage of 32 reduction
// indices the workgroup stages its S tile through LDS transposed (row-major,
// the 32 values of a row contiguous, hi then lo), splitting each FP32 value as
// it goes; each lane then reads the 8 consecutive reduction indices of one
// row that its MFMA operand needs.  The B fragments come split and transposed
// from Bs.  Tiles 128 x 128 (four wavefronts of 64 x 64), or 256 x 64 with
// the wavefronts stacked along the rows for ranks up to 64; the accumulator
// of a lane holds four consecutive rows of one column (one 16-byte store).
template <bool NARROW>
__global__ __launch_bounds__(256, 2) void lift_bf16_kernel(const LiftNode* __restrict__ nodes, int num_nodes) {
  constexpr int TMk = NARROW ? 4 * WT : TM;
  constexpr int TNk = NARROW ? WT : TN;
  constexpr int KS = 32;
  constexpr int RB = 144;             // LDS bytes per staged S row (64 hi, 64 lo, 16 pad)
  constexpr int RQ = TMk / 4;         // row quads of a tile
  constexpr int KC = KS * RQ / 256;   // columns per thread and stage (4 rows each)
  constexpr int KTS = 256;            // column-table chunk
  static_assert(KC * 256 == KS * RQ && (KC == 4 || KC == 8), "whole column quads per thread");
  typedef __attribute__((ext_vector_type(4))) int i4;

  const int item = xcd_item(blockIdx.x, gridDim.x);
  int lo = 0, hi = num_nodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].item_base <= item) lo = mid;
    else hi = mid - 1;
  }
  const LiftNode nd = nodes[lo];
  const int local = item - nd.item_base;
  const int rg = local / nd.col_tiles, ct = local % nd.col_tiles;
  const int64_t N = (nd.ncap > 0) ? min(*nd.rank, nd.ncap) : *nd.rank;
  if ((int64_t)ct * TNk >= N) return;  // whole workgroup
  const int rt_per = max(nd.rt_per, 1);
  const int rt_begin = rg * rt_per, rt_end = min(rt_begin + rt_per, nd.row_tiles);

  __shared__ __attribute__((aligned(16))) char sS[2][TMk * RB];
  __shared__ const char* tcol[KTS];
  __shared__ int64_t trbs[KTS];
  __shared__ int64_t trows[KTS];

  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int wi = NARROW ? wave : (wave >> 1), wj = NARROW ? 0 : (wave & 1);
  const int li = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)ct * TNk + wj * WT;
  const int m = nd.m;
  const int nks = (m + KS - 1) / KS;
  const int stages = nks;
  const int rq = t % RQ, kq = t / RQ;  // this thread's row quad and column group
  int table_base = -KTS;
  auto ensure_table = [&](int kfirst) {
    if (kfirst >= table_base && kfirst + KS <= table_base + KTS) return;
    __syncthreads();
    table_base = kfirst;
    const int k = kfirst + t;
    const bool kv = k < m;
    tcol[t] = kv ? reinterpret_cast<const char*>(nd.cols[k]) : nullptr;
    trbs[t] = kv ? nd.rbs[k] : kRowBlock;
    trows[t] = kv ? nd.crows[k] : 0;
    __syncthreads();
  };
  // this lane's B columns (one per 16-column block), zero past N
  const char* bcol[NB];
  bool bval[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t c = n0 + 16 * b + li;
    bval[b] = c < N;
    bcol[b] = nd.Bs + (bval[b] ? c : 0) * (int64_t)nks * 128 + 16 * g;
  }

  for (int rt = rt_begin; rt < rt_end; ++rt) {
    const int64_t rtile = (int64_t)rt * TMk;
    const bool active = (rtile + wi * WT < nd.n) && (n0 < N);
    f4 acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = f4{0, 0, 0, 0};
    // S runs of two stages in flight (wide tiles; the narrow ones have no
    // registers to spare and keep one)
    constexpr int NPS = NARROW ? 1 : 2;
    i4 psv[NPS][KC];
    bf8 ybh[NB], ybl[NB], nbh[NB], nbl[NB];
    auto gload_s = [&](int st, i4 (&ps)[KC]) {
      const int64_t row = rtile + 4 * rq;
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int k = st * KS + kq * KC + c;
        const int tk = k - table_base;
        const int64_t avail = (k < m) ? trows[tk] - row : 0;
        const float* p = (k < m) ? reinterpret_cast<const float*>(tcol[tk]) + (row >> 7) * trbs[tk] + (row & (kRowBlock - 1))
                                 : nullptr;
        if (avail >= 4 && (((uintptr_t)p & 15u) == 0)) {
          ps[c] = *(gptr<i4>)as_global(reinterpret_cast<const i4*>(p));
        } else {
          float x[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) x[e] = (e < avail) ? p[e] : 0.f;
          ps[c] = *reinterpret_cast<const i4*>(x);
        }
      }
    };
    auto gload_b = [&](int st, bf8 (&yh)[NB], bf8 (&yl)[NB]) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (bval[b]) {
          const char* q = bcol[b] + (int64_t)st * 128;
          yh[b] = *(gptr<bf8>)as_global(reinterpret_cast<const bf8*>(q));
          yl[b] = *(gptr<bf8>)as_global(reinterpret_cast<const bf8*>(q + 64));
        } else {
          yh[b] = __builtin_bit_cast(bf8, i4{0, 0, 0, 0});
          yl[b] = yh[b];
        }
      }
    };
    // rows 4 rq + e of columns kq KC .. kq KC + KC - 1, split into hi and lo
    auto lstore = [&](int buf, const i4 (&ps)[KC]) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t h[KC / 2], l[KC / 2];
#pragma unroll
        for (int c = 0; c < KC; c += 2)
          split_bf16x2(reinterpret_cast<const float*>(&ps[c])[e], reinterpret_cast<const float*>(&ps[c + 1])[e],
                       h[c / 2], l[c / 2]);
        char* q = sS[buf] + (4 * rq + e) * RB + kq * KC * 2;
        if constexpr (KC == 4) {
          typedef __attribute__((ext_vector_type(2))) int i2;
          *(i2*)q = i2{(int)h[0], (int)h[1]};
          *(i2*)(q + 64) = i2{(int)l[0], (int)l[1]};
        } else {
          *(i4*)q = i4{(int)h[0], (int)h[1], (int)h[2], (int)h[3]};
          *(i4*)(q + 64) = i4{(int)l[0], (int)l[1], (int)l[2], (int)l[3]};
        }
      }
    };
    auto compute = [&](int buf) {
      const char* sb = sS[buf] + (wi * WT + li) * RB + g * 16;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const bf8 xh = *(const bf8*)(sb + a * 16 * RB);
        const bf8 xl = *(const bf8*)(sb + a * 16 * RB + 64);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[a][b] = mfma_bf16(xl, ybh[b], acc[a][b]);
          acc[a][b] = mfma_bf16(xh, ybl[b], acc[a][b]);
          acc[a][b] = mfma_bf16(xh, ybh[b], acc[a][b]);
        }
      }
    };
    auto shift_b = [&]() {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        ybh[b] = nbh[b];
        ybl[b] = nbl[b];
      }
    };
    if constexpr (NPS == 1) {
      if (stages > 0) {
        ensure_table(0);
        gload_s(0, psv[0]);
        gload_b(0, ybh, ybl);
        lstore(0, psv[0]);
      }
      __syncthreads();
      for (int st = 0; st < stages; ++st) {
        const bool more = st + 1 < stages;
        if (more) {
          ensure_table((st + 1) * KS);
          gload_s(st + 1, psv[0]);
          gload_b(st + 1, nbh, nbl);
        }
        if (active) compute(st & 1);
        if (more) lstore((st + 1) & 1, psv[0]);
        __syncthreads();
        shift_b();
      }
    } else {
      // stage s sits in LDS buffer s & 1; while it is computed, stage s + 1
      // waits in registers (slot (s + 1) & 1) and stage s + 2 is loading
      // (slot s & 1); two stages per turn keep the slot indices constant
      if (stages > 0) {
        ensure_table(0);
        gload_s(0, psv[0]);
        gload_b(0, ybh, ybl);
        lstore(0, psv[0]);
        if (stages > 1) {
          ensure_table(KS);
          gload_s(1, psv[1]);
        }
      }
      __syncthreads();
      for (int st = 0; st < stages; st += 2) {
        if (st + 2 < stages) {
          ensure_table((st + 2) * KS);
          gload_s(st + 2, psv[0]);
        }
        if (st + 1 < stages) gload_b(st + 1, nbh, nbl);
        if (active) compute(0);
        if (st + 1 < stages) lstore(1, psv[1]);
        __syncthreads();
        shift_b();
        if (st + 1 >= stages) break;
        if (st + 3 < stages) {
          ensure_table((st + 3) * KS);
          gload_s(st + 3, psv[1]);
        }
        if (st + 2 < stages) gload_b(st + 2, nbh, nbl);
        if (active) compute(1);
        if (st + 2 < stages) lstore(0, psv[0]);
        __syncthreads();
        shift_b();
      }
    }
    if (!active) continue;
    float* out = reinterpret_cast<float*>(nd.out);
    const int64_t r0 = rtile + wi * WT;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t col = n0 + 16 * b + acc_col(lane);
      if (col >= N) continue;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int64_t row = r0 + 16 * a + acc_row<f4>(lane, 0);
        float* p = out + col * nd.ocs + blk_off(row, nd.obs);
        const f4 x = acc[a][b];
        if (row + 4 <= nd.n && (((uintptr_t)p & 15u) == 0)) {
          *(__attribute__((address_space(1))) fv4*)p = fv4{x[0], x[1], x[2], x[3]};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row + v < nd.n) p[v] = x[v];
        }
      }
    }
  }  // row tiles
}

// Bs from B32: one thread per (stage s, column c), c < N, consecutive
// threads on consecutive columns (rows of B32 read whole)
__global__ __launch_bounds__(256) void split_operand_kernel(const LiftNode* __restrict__ nodes) {
  const LiftNode nd = nodes[blockIdx.z];
  const int m = nd.m;
  const int nks = (m + 31) / 32;
  const int64_t N = (nd.ncap > 0) ? min(*nd.rank, nd.ncap) : *nd.rank;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nks) return;
  const int s = (int)(e / N);
  const int64_t c = e - (int64_t)s * N;
  uint32_t h[16], l[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = 32 * s + 2 * q;
    const float x0 = (k < m) ? nd.B32[(int64_t)k * nd.ldb + c] : 0.f;
    const float x1 = (k + 1 < m) ? nd.B32[(int64_t)(k + 1) * nd.ldb + c] : 0.f;
    split_bf16x2(x0, x1, h[q], l[q]);
  }
  typedef __attribute__((ext_vector_type(4))) unsigned u4;
  u4* dst = reinterpret_cast<u4*>(nd.Bs + (c * nks + s) * 128);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dst[q] = u4{h[4 * q], h[4 * q + 1], h[4 * q + 2], h[4 * q + 3]};
    dst[4 + q] = u4{l[4 * q], l[4 * q + 1], l[4 * q + 2], l[4 * q + 3]};
  }
}

}  // namespace

hapod_status launch_lift(int compute, const LiftNode* d_nodes, int num_nodes, int num_items,
                         hipStream_t stream, bool narrow) {
  if (num_items <= 0) return HAPOD_OK;
  const dim3 g(num_items), b(256);
  switch (compute * 2 + (narrow ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((lift_kernel<0, false>), g, b, 0, stream, d_nodes, num_nodes); break;
    case 1: hipLaunchKernelGGL((lift_kernel<0, true>), g, b, 0, stream, d_nodes, num_nodes); break;
    case 2: hipLaunchKernelGGL((lift_staged_kernel<1, false>), g, b, 0, stream, d_nodes, num_nodes); break;
    case 3: hipLaunchKernelGGL((lift_staged_kernel<1, true>), g, b, 0, stream, d_nodes, num_nodes); break;
    case 4: hipLaunchKernelGGL((lift_bf16_kernel<false>), g, b, 0, stream, d_nodes, num_nodes); break;
    case 5: hipLaunchKernelGGL((lift_bf16_kernel<true>), g, b, 0, stream, d_nodes, num_nodes); break;
    default: set_error("launch_lift: unknown compute mode"); return HAPOD_E_INVALID;
  }
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_split_operand(const LiftNode* d_nodes, int num_nodes, int64_t max_m, hipStream_t stream) {
  if (num_nodes <= 0 || max_m <= 0) return HAPOD_OK;
  const int64_t pairs = max_m * ((max_m + 31) / 32);
  hipLaunchKernelGGL(split_operand_kernel, dim3((unsigned)((pairs + 255) / 256), 1, (unsigned)num_nodes), dim3(256), 0,
                     stream, d_nodes);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_lift_dense(const LiftNode* d_nodes, int num_nodes, int num_items, hipStream_t stream) {
  if (num_items <= 0 || num_nodes <= 0) return HAPOD_OK;
  hipLaunchKernelGGL((lift_kernel<0, false, false, true>), dim3(num_items), dim3(256), 0, stream, d_nodes,
                     num_nodes);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_lift_residual(const LiftNode* d_node, int num_items, hipStream_t stream, bool dense) {
  if (num_items <= 0) return HAPOD_OK;
  if (dense)
    hipLaunchKernelGGL((lift_kernel<0, false, true, true>), dim3(num_items), dim3(256), 0, stream, d_node, 1);
  else
    hipLaunchKernelGGL((lift_kernel<0, false, true>), dim3(num_items), dim3(256), 0, stream, d_node, 1);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_sum_partials(const double* rpart, int64_t groups, int64_t N, double* res, hipStream_t stream) {
  if (N <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, rpart, groups, N,
                     res);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
