// Batched Gram matrices G = S^T S of the method of snapshots (Rem. 2.3).
//
// Work item = (node, upper tile pair (ti <= tj), row chunk).  Each
// wavefront accumulates a WT x WT block (WT = 16 NBW) as NBW x NBW MFMA
// blocks of 16 x 16.  Two arrangements:
//   tile 128 (quad): the four wavefronts own the four 64 x 64 quadrants of a
//     128 x 128 tile (NBW = 4) and stream every row of the chunk;
//   tile 64 / 32 / 16 (split): every wavefront computes the whole tile
//     (NBW = 4 / 2 / 1) over a quarter of the chunk's 128-row blocks, so a
//     narrow node still keeps all four SIMDs busy and the MFMA work is not
//     padded to 128 columns.
// The reduction index of the MFMA is the snapshot row, so every lane streams
// a contiguous run of rows of one column (column-major input): rows
// [k0 + R*g, k0 + R*g + R) of column c0 + l%16 for lane l = 16 g + l%16.
// Run element t feeds MFMA number t; the same row permutation is used for
// both operands, so the contraction is unchanged.
//
// Accumulation is in the MFMA's accumulator (FP64, or FP32 for the FP32 and
// split-BF16 forms); partial tiles (row chunks, and the wavefronts of a split
// tile) are summed in FP64 by gram_reduce in a fixed order, so results do not
// depend on scheduling.
#include "internal.hpp"
#include "mfma.hpp"

namespace hapod {
namespace {

template <int C> struct GramTraits;
// FP64 storage, FP64 MFMA 16x16x4: 4-row runs, 16 rows per batch
template <> struct GramTraits<0> { using Elem = double; using Acc = d4; static constexpr int R = 4; };
// FP32 storage, FP32 MFMA 16x16x4
template <> struct GramTraits<1> { using Elem = float; using Acc = f4; static constexpr int R = 4; };
// FP32 storage, split-BF16 MFMA 16x16x32 (8 rows per lane per MFMA)
template <> struct GramTraits<2> { using Elem = float; using Acc = f4; static constexpr int R = 8; };
// FP32 storage promoted to FP64, FP64 MFMA (used for double-accumulated
// Gram matrices of float data, e.g. re-orthonormalisation)
template <> struct GramTraits<3> { using Elem = float; using Acc = d4; static constexpr int R = 4; };

// Loads of one R-row run from a row-block-aligned global pointer (no guards).
template <int R, bool VEC>
__device__ __forceinline__ void run_full(gptr<double> p, double* out) {
  if constexpr (VEC) {
    const dv2 v0 = *(gptr<dv2>)(p);
    const dv2 v1 = *(gptr<dv2>)(p + 2);
    out[0] = v0[0]; out[1] = v0[1]; out[2] = v1[0]; out[3] = v1[1];
  } else {
#pragma unroll
    for (int t = 0; t < R; ++t) out[t] = p[t];
  }
}
template <int R, bool VEC>
__device__ __forceinline__ void run_full(gptr<float> p, float* out) {
  if constexpr (VEC) {
#pragma unroll
    for (int q = 0; q < R / 4; ++q) {
      const fv4 v = *(gptr<fv4>)(p + 4 * q);
      out[4 * q] = v[0]; out[4 * q + 1] = v[1]; out[4 * q + 2] = v[2]; out[4 * q + 3] = v[3];
    }
  } else {
#pragma unroll
    for (int t = 0; t < R; ++t) out[t] = p[t];
  }
}

template <int C, typename Acc, int R, int NBW>
__device__ __forceinline__ void mfma_batch(Acc (&acc)[NBW][NBW], typename GramTraits<C>::Elem (&va)[NBW][R],
                                           typename GramTraits<C>::Elem (&vb)[NBW][R]) {
  if constexpr (C == 0 || C == 3) {
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int a = 0; a < NBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) acc[a][b] = mfma_f64((double)va[a][t], (double)vb[b][t], acc[a][b]);
  } else if constexpr (C == 1) {
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int a = 0; a < NBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) acc[a][b] = mfma_f32(va[a][t], vb[b][t], acc[a][b]);
  } else {
    bf8 ha[NBW], la[NBW], hb[NBW], lb[NBW];
#pragma unroll
    for (int a = 0; a < NBW; ++a) {
      split_bf16x8(va[a], ha[a], la[a]);
      split_bf16x8(vb[a], hb[a], lb[a]);
    }
#pragma unroll
    for (int a = 0; a < NBW; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        acc[a][b] = mfma_bf16(la[a], hb[b], acc[a][b]);
        acc[a][b] = mfma_bf16(ha[a], lb[b], acc[a][b]);
        acc[a][b] = mfma_bf16(ha[a], hb[b], acc[a][b]);
      }
  }
}

// STAGED: the pre-split split-BF16 128 x 128 tile through LDS (every node of
// the launch pre-split); its own instantiation, so the register paths do not
// set its register budget.
template <int C, bool VEC, int NBW, bool QUAD, bool STAGED = false>
__global__ __launch_bounds__(256) void gram_tile_kernel(const GramNode* __restrict__ nodes,
                                                        const GramItem* __restrict__ items, int first) {
  static_assert(!STAGED || (C == 2 && QUAD && NBW == 4), "staged path: split-BF16 quad tiles only");
  using Tr = GramTraits<C>;
  using Elem = typename Tr::Elem;
  using Acc = typename Tr::Acc;
  constexpr int R = Tr::R;
  constexpr int KB = 4 * R;             // rows per MFMA batch
  constexpr int NBT = kRowBlock / KB;   // batches per 128-row block
  constexpr int WT = 16 * NBW;          // wavefront tile
  constexpr int TT = QUAD ? 2 * WT : WT;  // workgroup tile
  constexpr int BSTEP = QUAD ? 1 : 4;   // row blocks between a wavefront's blocks

  const GramItem item = items[first + xcd_item(blockIdx.x, gridDim.x)];
  const GramNode nd = nodes[item.node];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = QUAD ? (wave >> 1) : 0, wj = QUAD ? (wave & 1) : 0;
  const bool diag = (item.ti == item.tj);
  const int li = lane & 15, g = lane >> 4;
  const int cA0 = item.ti * TT + wi * WT, cB0 = item.tj * TT + wj * WT;
  // the lower sub-tile of a diagonal tile mirrors the upper one; sub-tiles
  // past m hold nothing
  const bool idle = (QUAD && diag && wi > wj) || cA0 >= nd.m || cB0 >= nd.m;
  // the staged path keeps every wavefront for its barriers
  constexpr bool kStaged = STAGED;
  if (idle && !kStaged) return;
  const bool same = (cA0 == cB0);  // both operands are the same columns

  // row range of this chunk; chunks start on 128-row block boundaries
  const int64_t r0 = (int64_t)item.chunk * nd.chunk_rows;
  const int64_t r1 = max(r0, min(min(nd.n, r0 + nd.chunk_rows), item.rlim));

  // column bases; columns past m alias the block's last column (their
  // products land in accumulator entries that are never stored)
  const Elem* pa[NBW];
  const Elem* pb[NBW];
  int64_t sa[NBW], sb[NBW], ra[NBW], rb[NBW];
#pragma unroll
  for (int a = 0; a < NBW; ++a) {
    const int ca = min(cA0 + a * 16 + li, nd.m - 1), cb = min(cB0 + a * 16 + li, nd.m - 1);
    pa[a] = reinterpret_cast<const Elem*>(nd.cols[ca]);
    pb[a] = reinterpret_cast<const Elem*>(nd.cols[cb]);
    sa[a] = nd.rbs[ca];
    sb[a] = nd.rbs[cb];
    ra[a] = nd.crows[ca];
    rb[a] = nd.crows[cb];
  }

  Acc acc[NBW][NBW];
#pragma unroll
  for (int a = 0; a < NBW; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  const int64_t blk0 = r0 >> 7, nblk = (r1 - r0 + kRowBlock - 1) >> 7;
  const int64_t bstart = QUAD ? 0 : wave;
  // the wavefront's blocks are bstart, bstart + BSTEP, ... < nblk
  const int64_t nwb = (bstart < nblk) ? (nblk - bstart + BSTEP - 1) / BSTEP : 0;
  if constexpr (kStaged) {
    {
      // Split-BF16, 128 x 128 tile: the workgroup stages 32 rows of its 256
      // columns (128 when ti = tj) through LDS as hi and lo bfloat16 runs,
      // double-buffered, so every value is fetched from global memory once
      // per workgroup instead of once per wavefront that reads it (two of
      // four); the next stage's loads are in flight while the current one
      // runs on the matrix cores.  Thread t always loads part t % 8 of a
      // column for columns 32 i + t / 8, i = 0..7: from a pre-split twin,
      // hi runs 0..3 or lo runs 4..7 of the 32-row step; from the FP32
      // columns, rows 4 part .. 4 part + 3, split into hi and lo as they go
      // to LDS (each value split once per workgroup; rows past a column's
      // own read as zero).  Same hi/lo pairs and products in the same order
      // as the register path below, so the sums are identical.
      constexpr int kColB = 8 * 16 + 16;  // LDS bytes per column and stage (padded)
      __shared__ __attribute__((aligned(16))) char stage[2][256 * kColB];
      const int t = threadIdx.x, part = t & 7;
      const int ncl = diag ? 128 : 256;  // columns staged
      const int nld = ncl / 32;          // loads per thread and stage
      const bool twin = nd.split != 0;
      const float* cp[8];
      int64_t cs[8], cr[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int cl = 32 * i + (t >> 3);
        const int base = (cl < 128) ? item.ti * TT + cl : item.tj * TT + (cl - 128);
        const int c = min(base, nd.m - 1);  // columns past m alias the last one
        cp[i] = reinterpret_cast<const float*>(nd.cols[c]);
        cs[i] = nd.rbs[c];
        cr[i] = nd.crows[c];
      }
      const int poff = (part < 4) ? part : 16 + (part - 4);  // bf8 offset in the step
      const int64_t S = nblk * NBT;  // 32-row steps of the chunk
      typedef __attribute__((ext_vector_type(4))) int i4;
      i4 pre[8];
      auto gload = [&](int64_t st) {
        const int64_t blk = blk0 + st / NBT;
        const int bt = (int)(st % NBT);
        if (twin) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < nld) pre[i] = ((gptr<i4>)as_global(cp[i] + blk * cs[i]))[4 * bt + poff];
        } else {
          const int roff = 32 * bt + 4 * part;  // row in the block
          const int64_t row = (blk << 7) + roff;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            if (i >= nld) continue;
            const float* p = cp[i] + blk * cs[i] + roff;
            const int64_t avail = cr[i] - row;
            if (avail >= 4 && (((uintptr_t)p & 15u) == 0)) {
              pre[i] = *(gptr<i4>)as_global(reinterpret_cast<const i4*>(p));
            } else {
              float x[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) x[e] = (e < avail) ? p[e] : 0.f;
              pre[i] = *reinterpret_cast<const i4*>(x);
            }
          }
        }
      };
      auto lstore = [&](int buf) {
        if (twin) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < nld) *(i4*)(stage[buf] + (32 * i + (t >> 3)) * kColB + part * 16) = pre[i];
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            if (i >= nld) continue;
            const float* x = reinterpret_cast<const float*>(&pre[i]);
            uint32_t h01, l01, h23, l23;
            split_bf16x2(x[0], x[1], h01, l01);
            split_bf16x2(x[2], x[3], h23, l23);
            char* q = stage[buf] + (32 * i + (t >> 3)) * kColB + part * 8;
            typedef __attribute__((ext_vector_type(2))) int i2;
            *(i2*)q = i2{(int)h01, (int)h23};
            *(i2*)(q + 64) = i2{(int)l01, (int)l23};
          }
        }
      };
      const int la = wi * 64, lb = diag ? wj * 64 : 128 + wj * 64;  // staged column bases
      auto compute = [&](int buf) {
        const char* sb = stage[buf];
        bf8 yh[NBW], yl[NBW];
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
          const char* q = sb + (lb + b * 16 + li) * kColB + g * 16;
          yh[b] = *(const bf8*)q;
          yl[b] = *(const bf8*)(q + 64);
        }
#pragma unroll
        for (int a = 0; a < NBW; ++a) {
          const char* q = sb + (la + a * 16 + li) * kColB + g * 16;
          const bf8 xh = *(const bf8*)q;
          const bf8 xl = *(const bf8*)(q + 64);
#pragma unroll
          for (int b = 0; b < NBW; ++b) {
            acc[a][b] = mfma_bf16(xl, yh[b], acc[a][b]);
            acc[a][b] = mfma_bf16(xh, yl[b], acc[a][b]);
            acc[a][b] = mfma_bf16(xh, yh[b], acc[a][b]);
          }
        }
      };
      if (S > 0) {
        gload(0);
        lstore(0);
      }
      __syncthreads();
      for (int64_t st = 0; st < S; ++st) {
        if (st + 1 < S) gload(st + 1);
        if (!idle) compute((int)(st & 1));
        if (st + 1 < S) lstore((int)((st + 1) & 1));
        __syncthreads();
      }
      if (idle) return;
    }
  } else {
  if constexpr (C == 2) {
    if (nd.split) {
      // pre-split columns: hi and lo bf16 runs straight from memory; blocks
      // are zero-padded past n, so every block is read whole.  Batches of
      // KB rows go through a two-deep register pipeline: the loads of batch
      // s + 1 are issued before the MFMAs of batch s, also across 128-row
      // blocks (the batches run in order, so the sums do not change).
      const int64_t S = nwb * NBT;
      bf8 xh[2][NBW], xl[2][NBW], yh[2][NBW], yl[2][NBW];
      auto ld = [&](int64_t st, int buf) {
        const int64_t blk = blk0 + bstart + (st / NBT) * BSTEP;
        const int bt = (int)(st % NBT);
#pragma unroll
        for (int a = 0; a < NBW; ++a) {
          gptr<bf8> ha = (gptr<bf8>)as_global(pa[a] + blk * sa[a]) + g;
          xh[buf][a] = ha[4 * bt];
          xl[buf][a] = ha[4 * bt + 16];
        }
        if (!QUAD && same) {
#pragma unroll
          for (int a = 0; a < NBW; ++a) {
            yh[buf][a] = xh[buf][a];
            yl[buf][a] = xl[buf][a];
          }
        } else {
#pragma unroll
          for (int a = 0; a < NBW; ++a) {
            gptr<bf8> hb = (gptr<bf8>)as_global(pb[a] + blk * sb[a]) + g;
            yh[buf][a] = hb[4 * bt];
            yl[buf][a] = hb[4 * bt + 16];
          }
        }
      };
      auto mm = [&](int buf) {
#pragma unroll
        for (int a = 0; a < NBW; ++a)
#pragma unroll
          for (int b = 0; b < NBW; ++b) {
            acc[a][b] = mfma_bf16(xl[buf][a], yh[buf][b], acc[a][b]);
            acc[a][b] = mfma_bf16(xh[buf][a], yl[buf][b], acc[a][b]);
            acc[a][b] = mfma_bf16(xh[buf][a], yh[buf][b], acc[a][b]);
          }
      };
      if (S > 0) ld(0, 0);
      for (int64_t st = 0; st < S; st += 2) {
        if (st + 1 < S) ld(st + 1, 1);
        mm(0);
        if (st + 1 < S) {
          if (st + 2 < S) ld(st + 2, 0);
          mm(1);
        }
      }
      goto store;
    }
  }
  {
  // 128-row blocks.  A block every column of the wavefront holds in full
  // runs unguarded at constant offsets; a block some column holds only in
  // part (its last one, or one past its rows) reads guarded.
  for (int64_t bi = bstart; bi < nblk; bi += BSTEP) {
    const int64_t blk = blk0 + bi;
    const int64_t rend = (blk + 1) << 7;
    int lane_full = 1;
#pragma unroll
    for (int a = 0; a < NBW; ++a) lane_full &= (ra[a] >= rend) & (rb[a] >= rend);
    if (__all(lane_full)) {
      gptr<Elem> qa[NBW], qb[NBW];
#pragma unroll
      for (int a = 0; a < NBW; ++a) {
        qa[a] = as_global(pa[a] + blk * sa[a] + R * g);
        qb[a] = as_global(pb[a] + blk * sb[a] + R * g);
      }
#pragma unroll
      for (int bt = 0; bt < NBT; ++bt) {
        Elem va[NBW][R], vb[NBW][R];
#pragma unroll
        for (int a = 0; a < NBW; ++a) run_full<R, VEC>(qa[a] + bt * KB, va[a]);
        if (!QUAD && same) {
#pragma unroll
          for (int a = 0; a < NBW; ++a)
#pragma unroll
            for (int t = 0; t < R; ++t) vb[a][t] = va[a][t];
        } else {
#pragma unroll
          for (int a = 0; a < NBW; ++a) run_full<R, VEC>(qb[a] + bt * KB, vb[a]);
        }
        mfma_batch<C, Acc, R, NBW>(acc, va, vb);
      }
    } else {
      for (int bt = 0; bt < NBT; ++bt) {
        const int64_t row = (blk << 7) + bt * KB + (int64_t)R * g;
        Elem va[NBW][R], vb[NBW][R];
#pragma unroll
        for (int a = 0; a < NBW; ++a) {
          const Elem* xa = pa[a] + blk * sa[a] + (row & (kRowBlock - 1));
          const Elem* xb = pb[a] + blk * sb[a] + (row & (kRowBlock - 1));
#pragma unroll
          for (int t = 0; t < R; ++t) {
            va[a][t] = (row + t < ra[a]) ? xa[t] : Elem(0);
            vb[a][t] = (row + t < rb[a]) ? xb[t] : Elem(0);
          }
        }
        mfma_batch<C, Acc, R, NBW>(acc, va, vb);
      }
    }
  }
  }
  }  // register paths

store:
  if (QUAD && nd.nchunks == 1) {
    // straight into G
#pragma unroll
    for (int a = 0; a < NBW; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row = cA0 + a * 16 + acc_row<Acc>(lane, v);
          int col = cB0 + b * 16 + acc_col(lane);
          if (nd.cross > 0) {
            if (row < nd.cross && col >= nd.cross && col < nd.m)
              nd.G[(int64_t)row * nd.ldg + (col - nd.cross)] = (double)acc[a][b][v];
          } else if (row < nd.m && col < nd.m && row <= col) {
            double x = (double)acc[a][b][v];
            nd.G[(int64_t)col * nd.ldg + row] = x;
            nd.G[(int64_t)row * nd.ldg + col] = x;
          }
        }
  } else {
    const int slot = ((item.pair - nd.pair_base) * nd.nchunks + item.chunk) * (QUAD ? 1 : 4) + (QUAD ? 0 : wave);
    double* P = nd.partial + (int64_t)slot * (TT * TT);
#pragma unroll
    for (int a = 0; a < NBW; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int i = wi * WT + a * 16 + acc_row<Acc>(lane, v);
          int j = wj * WT + b * 16 + acc_col(lane);
          P[j * TT + i] = (double)acc[a][b][v];
        }
  }
}

// Split-BF16 256 x 256 tiles of pre-split nodes: eight wavefronts, each a
// 128 x 64 block (8 x 4 MFMA blocks of 16 x 16), operands staged through LDS
// as in the 128-column staged path (32-row steps, double-buffered; one
// 512-thread workgroup per CU by its LDS).  Each value read from LDS feeds
// more products than with 64 x 64 quadrants (96 MFMAs per 24 fragment reads
// instead of 48 per 16), which relieves the LDS bandwidth that bounds the
// 128-column tiles.  Same products in the same order for every entry of G,
// so a row chunk's partial sums are those of the 128-column path.
// kTwin = false: a node of at most 256 columns (one diagonal tile pair) read
// from its own FP32 columns; each thread loads rows 4 part .. 4 part + 3 of
// a 32-row step of four columns and splits them into hi and lo as they go to
// LDS (rows past a column's own read as zero), as the 128-column staged path
// does, so every value leaves HBM once.
template <bool kTwin>
__global__ __launch_bounds__(512, 1) void gram_bf16_t256_kernel(const GramNode* __restrict__ nodes,
                                                                const GramItem* __restrict__ items, int first) {
  constexpr int TT = 256, NBA = 8, NBB = 4, NBT = kRowBlock / 32;
  constexpr int kColB = 8 * 16 + 16;  // LDS bytes per column and step (padded)
  const GramItem item = items[first + xcd_item(blockIdx.x, gridDim.x)];
  const GramNode nd = nodes[item.node];
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int wi = wave >> 2, wj = wave & 3;  // 128-row half, 64-column quarter
  const bool diag = (item.ti == item.tj);
  const int li = lane & 15, g = lane >> 4;
  const int cA0 = item.ti * TT + wi * 128, cB0 = item.tj * TT + wj * 64;
  // on a diagonal tile the blocks wholly below the diagonal mirror others
  const bool idle = (diag && wi * 128 >= wj * 64 + 64) || cA0 >= nd.m || cB0 >= nd.m;
  const int64_t r0 = (int64_t)item.chunk * nd.chunk_rows;
  const int64_t r1 = max(r0, min(min(nd.n, r0 + nd.chunk_rows), item.rlim));
  const int64_t blk0 = r0 >> 7, nblk = (r1 - r0 + kRowBlock - 1) >> 7;

  __shared__ __attribute__((aligned(16))) char stage[2][512 * kColB];
  typedef __attribute__((ext_vector_type(4))) int i4;
  const int part = t & 7;
  const int ncl = diag ? 256 : 512;  // columns staged
  const int nld = ncl / 64;          // loads per thread and step
  // the pre-split twin is row-block tiled: column c of block b at
  // base + b rbs + 128 c (one stride for all columns)
  const float* tw = reinterpret_cast<const float*>(nd.cols[0]);
  const int64_t trb = nd.rbs[0];
  const int poff = (part < 4) ? part : 16 + (part - 4);  // bf8 offset in the step
  const int64_t S = nblk * NBT;
  i4 pre[8];
  // FP32 columns (kTwin = false, diagonal tile of a node of <= 256 columns:
  // four columns per thread); their loads run two steps ahead (register
  // slots 0 and 1), the twin's one (it has no registers to spare)
  constexpr int kOwn = kTwin ? 1 : 4;
  i4 own[2][kOwn];
  const float* cp[kOwn];
  int64_t cs[kOwn], cr[kOwn];
  if constexpr (!kTwin) {
#pragma unroll
    for (int i = 0; i < kOwn; ++i) {
      const int c = min(item.ti * TT + 64 * i + (t >> 3), nd.m - 1);  // columns past m alias the last one
      cp[i] = reinterpret_cast<const float*>(nd.cols[c]);
      cs[i] = nd.rbs[c];
      cr[i] = nd.crows[c];
    }
  }
  auto gload = [&](int64_t st, int slot) {
    const int64_t blk = blk0 + st / NBT;
    const int bt = (int)(st % NBT);
    if constexpr (kTwin) {
      const float* bp = tw + blk * trb;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (i >= nld) continue;
        const int cl = 64 * i + (t >> 3);
        const int base = (cl < 256) ? item.ti * TT + cl : item.tj * TT + (cl - 256);
        const int c = min(base, nd.m - 1);  // columns past m alias the last one
        pre[i] = ((gptr<i4>)as_global(bp + (int64_t)c * kRowBlock))[4 * bt + poff];
      }
    } else {
      const int roff = 32 * bt + 4 * part;  // row in the block
      const int64_t row = (blk << 7) + roff;
#pragma unroll
      for (int i = 0; i < kOwn; ++i) {
        const float* p = cp[i] + blk * cs[i] + roff;
        const int64_t avail = cr[i] - row;
        i4 v;
        if (avail >= 4 && (((uintptr_t)p & 15u) == 0)) {
          v = *(gptr<i4>)as_global(reinterpret_cast<const i4*>(p));
        } else {
          float x[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) x[e] = (e < avail) ? p[e] : 0.f;
          v = *reinterpret_cast<const i4*>(x);
        }
        if (slot == 0) own[0][i] = v;
        else own[1][i] = v;
      }
    }
  };
  auto lstore = [&](int buf, int slot) {
    if constexpr (kTwin) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < nld) *(i4*)(stage[buf] + (64 * i + (t >> 3)) * kColB + part * 16) = pre[i];
    } else {
#pragma unroll
      for (int i = 0; i < kOwn; ++i) {
        const i4 v = (slot == 0) ? own[0][i] : own[1][i];
        const float* x = reinterpret_cast<const float*>(&v);
        uint32_t h01, l01, h23, l23;
        split_bf16x2(x[0], x[1], h01, l01);
        split_bf16x2(x[2], x[3], h23, l23);
        char* q = stage[buf] + (64 * i + (t >> 3)) * kColB + part * 8;
        typedef __attribute__((ext_vector_type(2))) int i2;
        *(i2*)q = i2{(int)h01, (int)h23};
        *(i2*)(q + 64) = i2{(int)l01, (int)l23};
      }
    }
  };
  f4 acc[NBA][NBB];
#pragma unroll
  for (int a = 0; a < NBA; ++a)
#pragma unroll
    for (int b = 0; b < NBB; ++b) acc[a][b] = f4{0, 0, 0, 0};
  const int la = wi * 128, lb = (diag ? 0 : 256) + wj * 64;
  auto compute = [&](int buf) {
    const char* sb = stage[buf];
    bf8 yh[NBB], yl[NBB];
#pragma unroll
    for (int b = 0; b < NBB; ++b) {
      const char* q = sb + (lb + b * 16 + li) * kColB + g * 16;
      yh[b] = *(const bf8*)q;
      yl[b] = *(const bf8*)(q + 64);
    }
#pragma unroll
    for (int a = 0; a < NBA; ++a) {
      const char* q = sb + (la + a * 16 + li) * kColB + g * 16;
      const bf8 xh = *(const bf8*)q;
      const bf8 xl = *(const bf8*)(q + 64);
#pragma unroll
      for (int b = 0; b < NBB; ++b) {
        acc[a][b] = mfma_bf16(xl, yh[b], acc[a][b]);
        acc[a][b] = mfma_bf16(xh, yl[b], acc[a][b]);
        acc[a][b] = mfma_bf16(xh, yh[b], acc[a][b]);
      }
    }
  };
  if constexpr (kTwin) {
    if (S > 0) {
      gload(0, 0);
      lstore(0, 0);
    }
    __syncthreads();
    for (int64_t st = 0; st < S; ++st) {
      if (st + 1 < S) gload(st + 1, 0);
      if (!idle) compute((int)(st & 1));
      if (st + 1 < S) lstore((int)((st + 1) & 1), 0);
      __syncthreads();
    }
  } else {
    // step s is staged in LDS buffer s & 1 from register slot s & 1; the
    // loop takes two steps per turn so every slot index is a constant
    if (S > 0) {
      gload(0, 0);
      if (S > 1) gload(1, 1);
      lstore(0, 0);
    }
    __syncthreads();
    for (int64_t st = 0; st < S; st += 2) {
      if (st + 2 < S) gload(st + 2, 0);
      if (!idle) compute(0);
      if (st + 1 < S) lstore(1, 1);
      __syncthreads();
      if (st + 1 >= S) break;
      if (st + 3 < S) gload(st + 3, 1);
      if (!idle) compute(1);
      if (st + 2 < S) lstore(0, 0);
      __syncthreads();
    }
  }
  if (idle) return;
  if (nd.nchunks == 1) {
#pragma unroll
    for (int a = 0; a < NBA; ++a)
#pragma unroll
      for (int b = 0; b < NBB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = cA0 + a * 16 + acc_row<f4>(lane, v);
          const int col = cB0 + b * 16 + acc_col(lane);
          if (row < nd.m && col < nd.m && row <= col) {
            const double x = (double)acc[a][b][v];
            nd.G[(int64_t)col * nd.ldg + row] = x;
            nd.G[(int64_t)row * nd.ldg + col] = x;
          }
        }
  } else {
    const int slot = (item.pair - nd.pair_base) * nd.nchunks + item.chunk;
    double* Pp = nd.partial + (int64_t)slot * (TT * TT);
#pragma unroll
    for (int a = 0; a < NBA; ++a)
#pragma unroll
      for (int b = 0; b < NBB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = wi * 128 + a * 16 + acc_row<f4>(lane, v);
          const int j = wj * 64 + b * 16 + acc_col(lane);
          Pp[j * TT + i] = (double)acc[a][b][v];
        }
  }
}

// Block-structured Gram: the tile pairs inside one child's diag(sigma^2)
// block, set rather than computed.  Grid: (fill, slice of 256 entries).
__global__ __launch_bounds__(256) void gram_fill_kernel(const GramFill* __restrict__ fills,
                                                        const double* __restrict__ s2) {
  const GramFill f = fills[blockIdx.x];
  const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (e >= (int64_t)f.rn * f.cn) return;
  const int i = (int)(e % f.rn), jj = (int)(e / f.rn);
  const int64_t row = f.r0 + i, col = f.c0 + jj;
  if (row > col) return;
  const double v = (row == col) ? s2[f.s2_off + row] : 0.0;
  f.G[col * f.ldg + row] = v;
  f.G[row * f.ldg + col] = v;
}

// Partial tiles of one tile pair summed in slot order (chunk, then
// wavefront), so the result does not depend on scheduling; the upper-triangle
// entries are written to both triangles of G.  Grid: (pair, slice of
// kReduceSlice tile entries); each thread keeps kReduceUnroll loads in flight.
constexpr int kReduceSlice = 256;
constexpr int kReduceUnroll = 8;

__global__ __launch_bounds__(kReduceSlice) void gram_reduce_kernel(const GramNode* __restrict__ nodes,
                                                                   const int32_t* __restrict__ pairs,
                                                                   const int32_t* __restrict__ pair_node) {
  const int node = pair_node[blockIdx.x];
  const int pair = pairs[blockIdx.x];
  const GramNode nd = nodes[node];
  const int TT = nd.tile;
  const int e = blockIdx.y * kReduceSlice + threadIdx.x;
  if (e >= TT * TT) return;
  const int lp = pair - nd.pair_base;
  int ti = 0, tj = 0;
  if (nd.cross > 0) {
    // cross product: compact (left tile, right tile) numbering
    const int tq = nd.cross / TT, nr = nd.ntiles - tq;
    ti = lp / nr;
    tj = tq + lp % nr;
  } else {
    // recover (ti, tj) from the local pair index in row-major upper order
    int rem = lp, rowlen = nd.ntiles;
    while (rem >= rowlen) { rem -= rowlen; ++ti; --rowlen; }
    tj = ti + rem;
  }
  const int i = e % TT, j = e / TT;
  const int row = ti * TT + i, col = tj * TT + j;
  if (row >= nd.m || col >= nd.m || row > col) return;
  const int ns = nd.nchunks * gram_slots_per_chunk(TT);
  const int64_t stride = (int64_t)TT * TT;
  const double* P = nd.partial + (int64_t)lp * ns * stride + e;
  double s = 0.0;
  int c = 0;
  for (; c + kReduceUnroll <= ns; c += kReduceUnroll) {
    double v[kReduceUnroll];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) v[u] = P[(int64_t)(c + u) * stride];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) s += v[u];
  }
  for (; c < ns; ++c) s += P[(int64_t)c * stride];
  if (nd.cross > 0) {
    nd.G[(int64_t)row * nd.ldg + (col - nd.cross)] = s;
    return;
  }
  nd.G[(int64_t)col * nd.ldg + row] = s;
  nd.G[(int64_t)row * nd.ldg + col] = s;
}

template <int C, bool VEC>
void launch_tile(int tile, const GramNode* d_nodes, const GramItem* d_items, int first, int count,
                 hipStream_t stream) {
  const dim3 g(count), b(256);
  switch (tile) {
    case 128: hipLaunchKernelGGL((gram_tile_kernel<C, VEC, 4, true>), g, b, 0, stream, d_nodes, d_items, first); break;
    case 64: hipLaunchKernelGGL((gram_tile_kernel<C, VEC, 4, false>), g, b, 0, stream, d_nodes, d_items, first); break;
    case 32: hipLaunchKernelGGL((gram_tile_kernel<C, VEC, 2, false>), g, b, 0, stream, d_nodes, d_items, first); break;
    default: hipLaunchKernelGGL((gram_tile_kernel<C, VEC, 1, false>), g, b, 0, stream, d_nodes, d_items, first); break;
  }
}

template <int C>
hapod_status launch_gram_c(const GramNode* d_nodes, const GramItem* d_items, const GramLaunch* launches,
                           int num_launches, hipStream_t stream) {
  for (int i = 0; i < num_launches; ++i) {
    const GramLaunch& L = launches[i];
    if (L.count <= 0) continue;
    if (L.tile != 256 && L.tile != 128 && L.tile != 64 && L.tile != 32 && L.tile != 16) {
      set_error("launch_gram: tile must be 256, 128, 64, 32 or 16");
      return HAPOD_E_INVALID;
    }
    if ((L.vec == 2 || L.vec == 3) && L.tile == 256) {
      if constexpr (C == 2) {
        if (L.vec == 2)
          hipLaunchKernelGGL(gram_bf16_t256_kernel<true>, dim3(L.count), dim3(512), 0, stream, d_nodes, d_items,
                             L.first);
        else
          hipLaunchKernelGGL(gram_bf16_t256_kernel<false>, dim3(L.count), dim3(512), 0, stream, d_nodes, d_items,
                             L.first);
      } else {
        set_error("launch_gram: 256-column tiles are split-BF16 only");
        return HAPOD_E_INVALID;
      }
    } else if (L.vec == 2) {
      if constexpr (C == 2) {
        if (L.tile != 128) {
          set_error("launch_gram: staged launches take 128-column tiles");
          return HAPOD_E_INVALID;
        }
        hipLaunchKernelGGL((gram_tile_kernel<2, true, 4, true, true>), dim3(L.count), dim3(256), 0, stream, d_nodes,
                           d_items, L.first);
      } else {
        set_error("launch_gram: staged launches are split-BF16 only");
        return HAPOD_E_INVALID;
      }
    } else if (L.vec) {
      launch_tile<C, true>(L.tile, d_nodes, d_items, L.first, L.count, stream);
    } else {
      launch_tile<C, false>(L.tile, d_nodes, d_items, L.first, L.count, stream);
    }
    HAPOD_HIP(hipGetLastError());
  }
  return HAPOD_OK;
}

}  // namespace

hapod_status launch_gram_fill(const GramFill* d_fills, int count, const double* s2_base, hipStream_t stream) {
  if (count <= 0) return HAPOD_OK;
  // tiles are at most 256 x 256
  hipLaunchKernelGGL(gram_fill_kernel, dim3((unsigned)count, 256), dim3(256), 0, stream, d_fills, s2_base);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_gram(int compute, const GramNode* d_nodes, const GramItem* d_items,
                         const GramLaunch* launches, int num_launches,
                         const int32_t* d_reduce_pairs, const int32_t* d_reduce_node, int num_reduce,
                         int max_tile, hipStream_t stream) {
  for (int i = 0; i < num_launches; ++i) {
    const int c = launches[i].compute >= 0 ? launches[i].compute : compute;
    switch (c) {
      case 0: HAPOD_TRY(launch_gram_c<0>(d_nodes, d_items, launches + i, 1, stream)); break;
      case 1: HAPOD_TRY(launch_gram_c<1>(d_nodes, d_items, launches + i, 1, stream)); break;
      case 2: HAPOD_TRY(launch_gram_c<2>(d_nodes, d_items, launches + i, 1, stream)); break;
      case 3: HAPOD_TRY(launch_gram_c<3>(d_nodes, d_items, launches + i, 1, stream)); break;
      default: set_error("launch_gram: unknown compute mode"); return HAPOD_E_INVALID;
    }
  }
  if (num_reduce > 0) {
    const unsigned slices = (unsigned)((max_tile * max_tile + kReduceSlice - 1) / kReduceSlice);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(num_reduce, slices), dim3(kReduceSlice), 0, stream, d_nodes,
                       d_reduce_pairs, d_reduce_node);
    HAPOD_HIP(hipGetLastError());
  }
  return HAPOD_OK;
}

}  // namespace hapod
