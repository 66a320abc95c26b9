// Batched symmetric eigensolver for Gram matrices (Rem. 2.3), FP64,
// one workgroup per matrix: parallel cyclic two-sided Jacobi.
//
// Ordering: round-robin tournament.  The m2 = m + (m odd) indices sit in
// slots; slots (2k, 2k+1) form pair k, so every round rotates h = m2/2
// disjoint pairs at once.  After a round all data moves to the next slot
// arrangement (slot 0 fixed, the others circulate), so that after m2 - 1
// rounds every pair of indices has met exactly once (one sweep).  The move is
// fused into the update: each 2 x 2 block (pair P rows, pair Q columns) is
// read from the current buffer, rotated on both sides, and written to its
// permuted place in the other buffer.  Only the upper triangle is stored, so
// the matrix stays exactly symmetric.
//
// Rotation (Golub & Van Loan, symmetric Schur 2 x 2): tau = (a_qq - a_pp) /
// (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1+t^2),
// s = t c; a_pp' = a_pp - t a_pq, a_qq' = a_qq + t a_pq, a_pq' = 0.  A pair
// is skipped when |a_pq| <= max(tol * sqrt(|a_pp a_qq|), 2^-60 max|diag|);
// iteration stops after a sweep without rotations.
//
// Output: eigenvalues descending (ties by original index), eigenvector
// columns with their largest-magnitude entry made positive.
#include "internal.hpp"

namespace hapod {
namespace {

constexpr int kThreads = 256;         // LDS variant (m <= 128)
constexpr int kThreadsGlobal = 1024;  // global variant: more loads in flight per round
constexpr int kMaxSweeps = 60;
constexpr double kTolRel = 1e-14;

__device__ __forceinline__ int slot_next(int s, int h) {
  if (h == 1 || s == 0) return s;
  if ((s & 1) == 0) {
    int k = s >> 1;
    return (k <= h - 2) ? 2 * (k + 1) : 2 * (h - 1) + 1;
  }
  int k = (s - 1) >> 1;
  return (k == 0) ? 2 : 2 * (k - 1) + 1;
}

// The two buffers are picked with a select, not by indexing a two-entry
// array: a dynamically indexed array would live in per-lane scratch memory.
struct GlobalStore {
  double* buf[2];
  int ld;
  __device__ __forceinline__ double& at(int b, int i, int j) const {  // i <= j
    return (b ? buf[1] : buf[0])[(int64_t)j * ld + i];
  }
};
struct LdsStore {
  double* buf[2];
  __device__ __forceinline__ double& at(int b, int i, int j) const {  // i <= j
    return (b ? buf[1] : buf[0])[(j * (j + 1) >> 1) + i];
  }
};

template <class Store>
__device__ void jacobi_body(const EigNode& nd, Store st, double* cs, double* sn, double* tn,
                            int* label0, int* label1, int* nrot_sh, double* red) {
  const int m = nd.m;
  const int m2 = m + (m & 1);
  const int h = m2 >> 1;
  const int tid = threadIdx.x;
  double* V0 = nd.Vwork;
  double* V1 = nd.Vwork + (int64_t)m * m2;

  // ---- load upper triangle, zero the padding slot, V = I -----------------
  for (int64_t e = tid; e < (int64_t)m2 * m2; e += blockDim.x) {
    int i = (int)(e % m2), j = (int)(e / m2);
    if (i > j) continue;
    double x = (i < m && j < m) ? nd.G[(int64_t)j * nd.ldg + i] : 0.0;
    st.at(0, i, j) = x;
  }
  for (int64_t e = tid; e < (int64_t)m * m2; e += blockDim.x) {
    int r = (int)(e % m), s = (int)(e / m);
    V0[e] = (r == s) ? 1.0 : 0.0;
  }
  for (int s = tid; s < m2; s += blockDim.x) label0[s] = s;
  // max |diag| for the absolute skip threshold
  double dmax = 0.0;
  for (int i = tid; i < m; i += blockDim.x) dmax = fmax(dmax, fabs(nd.G[(int64_t)i * nd.ldg + i]));
  red[tid] = dmax;
  __syncthreads();
  for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double tol_abs = ldexp(red[0], -60);
  __syncthreads();

  int cur = 0;
  int* lab[2] = {label0, label1};
  int executed = 0;
  const int rounds = (m2 > 1) ? m2 - 1 : 0;
  const int nblk = h * (h + 1) / 2;
  for (int sweep = 0; sweep < kMaxSweeps && m > 1; ++sweep) {
    ++executed;
    if (tid == 0) *nrot_sh = 0;
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
      const int nxt = cur ^ 1;
      // phase 1: rotation of every pair
      int local_rot = 0;
      for (int k = tid; k < h; k += blockDim.x) {
        const int p = 2 * k, q = p + 1;
        double c = 1.0, s = 0.0, t = 0.0;
        if (lab[cur][p] < m && lab[cur][q] < m) {
          const double app = st.at(cur, p, p), aqq = st.at(cur, q, q), apq = st.at(cur, p, q);
          const double thr = fmax(kTolRel * sqrt(fabs(app * aqq)), tol_abs);
          if (fabs(apq) > thr) {
            const double tau = (aqq - app) / (2.0 * apq);
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            ++local_rot;
          }
        }
        cs[k] = c; sn[k] = s; tn[k] = t;
      }
      if (local_rot) atomicAdd(nrot_sh, local_rot);
      __syncthreads();
      // phase 2: two-sided update of the 2 x 2 blocks, written permuted
      for (int idx = tid; idx < nblk; idx += blockDim.x) {
        int Q = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while ((Q + 1) * (Q + 2) / 2 <= idx) ++Q;
        while (Q * (Q + 1) / 2 > idx) --Q;
        const int P = idx - Q * (Q + 1) / 2;
        const int p0 = 2 * P, p1 = p0 + 1, q0 = 2 * Q, q1 = q0 + 1;
        const int sp0 = slot_next(p0, h), sp1 = slot_next(p1, h);
        if (P == Q) {
          const double app = st.at(cur, p0, p0), aqq = st.at(cur, p1, p1), apq = st.at(cur, p0, p1);
          const double t = tn[P];
          st.at(nxt, sp0, sp0) = app - t * apq;
          st.at(nxt, sp1, sp1) = aqq + t * apq;
          st.at(nxt, min(sp0, sp1), max(sp0, sp1)) = (t != 0.0) ? 0.0 : apq;
          continue;
        }
        const double b00 = st.at(cur, p0, q0), b01 = st.at(cur, p0, q1);
        const double b10 = st.at(cur, p1, q0), b11 = st.at(cur, p1, q1);
        const double cP = cs[P], sP = sn[P], cQ = cs[Q], sQ = sn[Q];
        const double l00 = cP * b00 - sP * b10, l01 = cP * b01 - sP * b11;
        const double l10 = sP * b00 + cP * b10, l11 = sP * b01 + cP * b11;
        const double n00 = cQ * l00 - sQ * l01, n01 = sQ * l00 + cQ * l01;
        const double n10 = cQ * l10 - sQ * l11, n11 = sQ * l10 + cQ * l11;
        const int sq0 = slot_next(q0, h), sq1 = slot_next(q1, h);
        st.at(nxt, min(sp0, sq0), max(sp0, sq0)) = n00;
        st.at(nxt, min(sp0, sq1), max(sp0, sq1)) = n01;
        st.at(nxt, min(sp1, sq0), max(sp1, sq0)) = n10;
        st.at(nxt, min(sp1, sq1), max(sp1, sq1)) = n11;
      }
      // phase 3: eigenvector columns, permuted the same way
      {
        double* Vc = cur ? V1 : V0;
        double* Vn = cur ? V0 : V1;
        for (int64_t e = tid; e < (int64_t)m * h; e += blockDim.x) {
          const int row = (int)(e % m), P = (int)(e / m);
          const double vp = Vc[(int64_t)(2 * P) * m + row], vq = Vc[(int64_t)(2 * P + 1) * m + row];
          const double c = cs[P], s = sn[P];
          Vn[(int64_t)slot_next(2 * P, h) * m + row] = c * vp - s * vq;
          Vn[(int64_t)slot_next(2 * P + 1, h) * m + row] = s * vp + c * vq;
        }
      }
      for (int s = tid; s < m2; s += blockDim.x) lab[nxt][slot_next(s, h)] = lab[cur][s];
      __syncthreads();
      cur = nxt;
    }
    const int nrot = *nrot_sh;
    __syncthreads();
    if (nrot == 0) break;
  }

  // ---- sort descending (ties by original index), sign fix, write ---------
  const double* Vf = cur ? V1 : V0;
  for (int s = tid; s < m2; s += blockDim.x) {
    const int ls = lab[cur][s];
    if (ls >= m) continue;
    const double lam = st.at(cur, s, s);
    int rank = 0;
    for (int s2 = 0; s2 < m2; ++s2) {
      const int l2 = lab[cur][s2];
      if (l2 >= m || s2 == s) continue;
      const double x = st.at(cur, s2, s2);
      if (x > lam || (x == lam && l2 < ls)) ++rank;
    }
    // sign: largest |entry| positive (first one on ties)
    const double* col = Vf + (int64_t)s * m;
    double best = -1.0, sgn = 1.0;
    for (int rr = 0; rr < m; ++rr) {
      const double a = fabs(col[rr]);
      if (a > best) { best = a; sgn = (col[rr] < 0.0) ? -1.0 : 1.0; }
    }
    nd.lambda[rank] = lam;
    double* out = nd.V + (int64_t)rank * nd.ldv;
    for (int rr = 0; rr < m; ++rr) out[rr] = sgn * col[rr];
  }
  if (tid == 0 && nd.sweeps) *nd.sweeps = executed;
}

__global__ __launch_bounds__(kThreadsGlobal) void jacobi_global_kernel(const EigNode* __restrict__ nodes) {
  __shared__ double cs[kJacobiMax / 2], sn[kJacobiMax / 2], tn[kJacobiMax / 2];
  __shared__ int lab0[kJacobiMax], lab1[kJacobiMax];
  __shared__ int nrot;
  __shared__ double red[kThreadsGlobal];
  const EigNode nd = nodes[blockIdx.x];
  if (nd.m <= 0) return;
  const int m2 = nd.m + (nd.m & 1);
  GlobalStore st;
  st.buf[0] = nd.work;
  st.buf[1] = nd.work + (int64_t)m2 * m2;
  st.ld = m2;
  jacobi_body(nd, st, cs, sn, tn, lab0, lab1, &nrot, red);
}

constexpr int kPackedMax = kJacobiLdsMax * (kJacobiLdsMax + 1) / 2;

__global__ __launch_bounds__(kThreads) void jacobi_lds_kernel(const EigNode* __restrict__ nodes) {
  extern __shared__ double lds[];
  __shared__ double cs[kJacobiLdsMax / 2], sn[kJacobiLdsMax / 2], tn[kJacobiLdsMax / 2];
  __shared__ int lab0[kJacobiLdsMax], lab1[kJacobiLdsMax];
  __shared__ int nrot;
  __shared__ double red[kThreads];
  const EigNode nd = nodes[blockIdx.x];
  if (nd.m <= 0) return;
  LdsStore st;
  st.buf[0] = lds;
  st.buf[1] = lds + kPackedMax;
  jacobi_body(nd, st, cs, sn, tn, lab0, lab1, &nrot, red);
}

}  // namespace

size_t jacobi_work_doubles(int m) {
  const size_t m2 = (size_t)(m + (m & 1));
  return 2 * m2 * m2;
}
size_t jacobi_vwork_doubles(int m) {
  const size_t m2 = (size_t)(m + (m & 1));
  return 2 * (size_t)m * m2;
}

hapod_status launch_jacobi(const EigNode* d_nodes, int num_nodes, int max_m, hipStream_t stream) {
  if (num_nodes <= 0) return HAPOD_OK;
  if (max_m > kJacobiMax) {
    set_error("launch_jacobi: m above the Jacobi limit");
    return HAPOD_E_UNSUPPORTED;
  }
  if (max_m <= kJacobiLdsMax) {
    const size_t lds = 2 * kPackedMax * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      HAPOD_HIP(hipFuncSetAttribute((const void*)jacobi_lds_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      attr_set = true;
    }
    hipLaunchKernelGGL(jacobi_lds_kernel, dim3(num_nodes), dim3(kThreads), lds, stream, d_nodes);
  } else {
    hipLaunchKernelGGL(jacobi_global_kernel, dim3(num_nodes), dim3(kThreadsGlobal), 0, stream, d_nodes);
  }
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
