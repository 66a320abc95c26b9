// Gram matrix G = S^T S (Rem. 2.3) without any device allocation, for callers
// that cannot allocate (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc): the descriptors and the partial tiles of
// the row chunks live in one file-scope device array, `scratch`, written by a
// set-up kernel from scalar arguments (no host staging either), then the
// library's Gram kernels run on it exactly as hapod_gram runs them, with the
// number of row chunks capped so the partial tiles fit.
//
// Every call on a device shares that device's array and leaves its last
// contents there; nothing in it needs to start at zero (every descriptor and
// every partial slot a call reads, the same call wrote first).  Calls that
// overlap on one device (two streams, two threads) race on it.
#include <mutex>

#include "internal.hpp"

namespace hapod {
namespace {

// Partial tiles: at most 64 MiB (for m <= 256: 3 tile pairs x 128 chunks x
// 128^2 doubles, or one 256^2 pair x 128 chunks); descriptors below 256 KiB.
constexpr size_t kPartialBytes = size_t(64) << 20;
constexpr size_t kDescBytes = size_t(256) << 10;
constexpr size_t kScratchBytes = kDescBytes + kPartialBytes;
constexpr int64_t kNoAllocMaxM = 256;
constexpr int kMaxChunks = 128;

__device__ __align__(256) char scratch[kScratchBytes];

// Descriptor layout inside the array (byte offsets).
constexpr size_t kOffCols = 0;                                   // m column pointers
constexpr size_t kOffRbs = kOffCols + sizeof(void*) * kNoAllocMaxM;
constexpr size_t kOffRows = kOffRbs + sizeof(int64_t) * kNoAllocMaxM;
constexpr size_t kOffNode = kOffRows + sizeof(int64_t) * kNoAllocMaxM;
constexpr size_t kOffPairs = kOffNode + 256;                      // reduce pair list
constexpr size_t kOffPairNode = kOffPairs + sizeof(int32_t) * 64;
constexpr size_t kOffItems = kOffPairNode + sizeof(int32_t) * 64;  // work items
static_assert(kOffItems + sizeof(GramItem) * 64 * kMaxChunks <= kDescBytes, "descriptors fit");
static_assert(sizeof(GramNode) <= 256, "node fits");

// One workgroup: column table (S plain, ld lds), the node, the work items
// (tile pairs in row-major upper order, each with its nchunks row chunks, as
// hapod_gram orders them) and the reduce list.
__global__ __launch_bounds__(256) void noalloc_setup_kernel(char* base, const char* S, int64_t col_bytes, int32_t m,
                                                            int64_t n, int32_t tile, int32_t nchunks,
                                                            int64_t chunk_rows, double* G, int64_t ldg, int32_t slots) {
  const void** cols = reinterpret_cast<const void**>(base + kOffCols);
  int64_t* rbs = reinterpret_cast<int64_t*>(base + kOffRbs);
  int64_t* rows = reinterpret_cast<int64_t*>(base + kOffRows);
  const int nt = (m + tile - 1) / tile;
  const int pairs = nt * (nt + 1) / 2;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    cols[j] = S + (int64_t)j * col_bytes;
    rbs[j] = kRowBlock;
    rows[j] = n;
  }
  GramItem* items = reinterpret_cast<GramItem*>(base + kOffItems);
  for (int idx = threadIdx.x; idx < pairs * nchunks; idx += blockDim.x) {
    const int p = idx / nchunks, c = idx - p * nchunks;
    int ti = 0, rem = p, rowlen = nt;
    while (rem >= rowlen) {
      rem -= rowlen;
      ++ti;
      --rowlen;
    }
    GramItem it;
    it.node = 0;
    it.ti = (int16_t)ti;
    it.tj = (int16_t)(ti + rem);
    it.chunk = c;
    it.pair = p;
    it.rlim = INT64_MAX;
    items[idx] = it;
  }
  int32_t* rp = reinterpret_cast<int32_t*>(base + kOffPairs);
  int32_t* rn = reinterpret_cast<int32_t*>(base + kOffPairNode);
  for (int p = threadIdx.x; p < pairs; p += blockDim.x) {
    rp[p] = p;
    rn[p] = 0;
  }
  if (threadIdx.x == 0) {
    GramNode g{};
    g.cols = cols;
    g.rbs = rbs;
    g.crows = rows;
    g.split = 0;
    g.n = n;
    g.chunk_rows = chunk_rows;
    g.G = G;
    g.partial = slots > 1 ? reinterpret_cast<double*>(base + kDescBytes) : nullptr;
    g.ldg = ldg;
    g.m = m;
    g.nchunks = nchunks;
    g.ntiles = nt;
    g.pair_base = 0;
    g.tile = tile;
    g.cross = 0;
    *reinterpret_cast<GramNode*>(base + kOffNode) = g;
  }
}

__global__ __launch_bounds__(256) void zero_square_kernel(double* G, int64_t ldg, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  G[(e / m) * ldg + e % m] = 0.0;
}

// Device address of `scratch` on each device, looked up once per device with
// that device current.  In host code the array's name is only a host-side
// stand-in: kernels get this address, never the name.
constexpr int kMaxDevices = 64;
char* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

hapod_status scratch_for_current_device(char** out) {
  int dev = 0;
  HAPOD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("hapod_gram_noalloc: device index beyond 64");
    return HAPOD_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hapod_gram_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                hipGetErrorString(e));
      return HAPOD_E_DEVICE;
    }
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return HAPOD_OK;
}

}  // namespace
}  // namespace hapod

using namespace hapod;

extern "C" hapod_status hapod_gram_noalloc(hapod_precision prec, int64_t n, int64_t m, const void* S, int64_t lds,
                                           double* G, int64_t ldg, void* stream_) {
  if (prec != HAPOD_FP64 && prec != HAPOD_FP32 && prec != HAPOD_BF16X3) {
    set_error("hapod_gram_noalloc: unknown precision");
    return HAPOD_E_INVALID;
  }
  if (n < 0 || m < 0 || (m > 0 && (!G || (n > 0 && !S))) || lds < std::max<int64_t>(n, 1) ||
      ldg < std::max<int64_t>(m, 1)) {
    set_error("hapod_gram_noalloc: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (m > kNoAllocMaxM) {
    set_error("hapod_gram_noalloc: m = " + std::to_string(m) + " exceeds the 256 columns its scratch array holds");
    return HAPOD_E_UNSUPPORTED;
  }
  if (m == 0) return HAPOD_OK;
  hipStream_t stream = (hipStream_t)stream_;
  char* base = nullptr;
  HAPOD_TRY(scratch_for_current_device(&base));
  if (n == 0) {
    hipLaunchKernelGGL(zero_square_kernel, dim3((unsigned)((m * m + 255) / 256)), dim3(256), 0, stream, G, ldg, m);
    HAPOD_HIP(hipGetLastError());
    return HAPOD_OK;
  }
  const int compute = prec == HAPOD_FP64 ? 0 : (prec == HAPOD_FP32 ? 1 : 2);
  const int eb = prec == HAPOD_FP64 ? 8 : 4;
  // the tiles hapod_gram takes for m <= 256: split-BF16 above 128 columns one
  // 256-column tile staged from the FP32 columns, from 65 columns 128-column
  // tiles split while staged, narrower nodes on FP32 MFMA
  int tile = gram_tile_for(m);
  const bool own256 = (compute == 2 && tile == 128 && m > 128);
  if (own256) tile = 256;
  const int gc = (compute == 2 && m < kBf16MinCols) ? 1 : compute;
  const int nt = (int)((m + tile - 1) / tile);
  const int pairs = nt * (nt + 1) / 2;
  const int spc = gram_slots_per_chunk(tile);
  const int KB = (compute == 2) ? 32 : 16;
  // row chunks as hapod_gram picks them, capped so that the partial tiles fit
  const int64_t per_chunk = (int64_t)pairs * spc * tile * tile * (int64_t)sizeof(double);
  const int cap = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxChunks, (int64_t)kPartialBytes / per_chunk));
  int nch = std::min(cap, pick_chunks(n, pairs, std::max(8192, pairs), 2048));
  const int64_t cr = ((n + nch - 1) / nch + kRowBlock - 1) / kRowBlock * kRowBlock;
  nch = (int)((n + cr - 1) / cr);
  const int slots = nch * spc;
  bool vec_ok = (cr % KB == 0) && (((uintptr_t)S & 15u) == 0) && ((lds * eb) % 16 == 0);
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(256), 0, stream, base, (const char*)S, lds * eb, (int32_t)m, n,
                     (int32_t)tile, (int32_t)nch, cr, G, ldg, (int32_t)slots);
  HAPOD_HIP(hipGetLastError());
  const int vec_mode = own256 ? 3 : (gc == 2 && tile >= 128) ? 2 : (vec_ok ? 1 : 0);
  const GramLaunch gl{tile, vec_mode, 0, (int32_t)(pairs * nch), gc != compute ? gc : -1};
  return launch_gram(compute, reinterpret_cast<const GramNode*>(base + kOffNode),
                     reinterpret_cast<const GramItem*>(base + kOffItems), &gl, 1,
                     reinterpret_cast<const int32_t*>(base + kOffPairs),
                     reinterpret_cast<const int32_t*>(base + kOffPairNode), slots > 1 ? pairs : 0, tile, stream);
}
