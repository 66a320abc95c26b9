// C ABI of the HAPOD library: step-level entry points, the plan (tree
// validation, levels, Thm. 3.5 tolerances) and the level scheduler.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <functional>
#include <vector>

#include "internal.hpp"
#include "wide.hpp"

namespace hapod {

namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }

void* pool_alloc_cb(void* pool, size_t bytes);
void pool_free_cb(void* pool, void* p);
hapod_status gram_impl(int compute, int eb, int64_t n, int64_t m, const void* S, int64_t lds, double* G, int64_t ldg,
                       hipStream_t stream, int tile = 0, int64_t in_rbs = 0);

int pick_chunks(int64_t n, int pairs, int target_items, int64_t min_rows) {
  int64_t want = std::max<int64_t>(1, (target_items + pairs - 1) / pairs);
  int64_t maxc = std::max<int64_t>(1, n / std::max<int64_t>(min_rows, 1));
  return (int)std::max<int64_t>(1, std::min(want, maxc));
}

// Gram tile for a node of m columns: narrow nodes get split tiles (every
// wavefront of a workgroup on the whole tile, over its own rows) sized to m,
// so their MFMA work is not padded to 128 columns and no SIMD idles.
int gram_tile_for(int64_t m) {
  if (m <= 16) return 16;
  if (m <= 32) return 32;
  if (m <= 64) return 64;
  return kGramTile;
}

namespace {

int elem_bytes(hapod_precision p) { return p == HAPOD_FP64 ? 8 : 4; }
int compute_mode(hapod_precision p) { return p == HAPOD_FP64 ? 0 : (p == HAPOD_FP32 ? 1 : 2); }

constexpr size_t kAlign = 256;
constexpr int kSuperI = 4, kSuperJ = 8;  // Gram tile pairs per super-tile (32 = CUs of an XCD)

// plain column-major n x m (leading dimension ld)
std::vector<const void*> column_table(const void* base, int64_t ld, int64_t m, int eb) {
  std::vector<const void*> v((size_t)m);
  for (int64_t j = 0; j < m; ++j) v[j] = (const char*)base + j * ld * eb;
  return v;
}
// row-block-tiled n x m_cap buffer: column j starts kRowBlock * j elements in
int64_t tiled_rbs(int64_t m_cap) { return m_cap * kRowBlock; }
std::vector<const void*> tiled_table(const void* base, int64_t m, int eb) {
  std::vector<const void*> v((size_t)m);
  for (int64_t j = 0; j < m; ++j) v[j] = (const char*)base + j * kRowBlock * eb;
  return v;
}
size_t tiled_bytes(int64_t n, int64_t m_cap, int eb) {
  return (size_t)((n + kRowBlock - 1) / kRowBlock) * kRowBlock * m_cap * eb;
}
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// Device memory pool: exact-size reuse of freed blocks, so repeated runs of
// the same plan allocate nothing after the first; an optional cap on the
// bytes held.
// ---------------------------------------------------------------------------
class Pool {
 public:
  static constexpr size_t kBestFitMin = size_t(256) << 20;
  static constexpr size_t kReserve = size_t(2) << 30;
  ~Pool() { release_all(); }
  hapod_status alloc(size_t bytes, void** out) {
    bytes = align_up(std::max<size_t>(bytes, kAlign));
    auto it = free_.find(bytes);
    if (it != free_.end() && !it->second.empty()) {
      *out = it->second.back();
      it->second.pop_back();
      return HAPOD_OK;
    }
    // a large request may take the smallest cached block of up to twice its
    // size: mapping fresh device memory costs about 20 ms per GiB, so reusing
    // a held block beats returning it and allocating anew
    if (bytes >= kBestFitMin)
      for (auto jt = free_.lower_bound(bytes); jt != free_.end() && jt->first <= 2 * bytes; ++jt)
        if (!jt->second.empty()) {
          *out = jt->second.back();
          jt->second.pop_back();
          return HAPOD_OK;
        }
    if (cap_ && held_ + bytes > cap_) {
      // give cached blocks back before failing
      trim();
      if (held_ + bytes > cap_) {
        set_error("device memory cap exceeded: need " + std::to_string(held_ + bytes) + " bytes, cap " +
                  std::to_string(cap_));
        return HAPOD_E_NOMEM;
      }
    }
    // keep some device memory free for the runtime and the caller: below
    // that, cached blocks go back (largest first, only as many as needed)
    // before mapping more
    size_t fr = 0, tot = 0;
    if (!free_.empty() && hipMemGetInfo(&fr, &tot) == hipSuccess && fr < bytes + kReserve)
      trim_until(bytes + kReserve - fr);
    void* p = nullptr;
    if (verbose_) std::fprintf(stderr, "[hapod pool] map %zu bytes (free %zu)\n", bytes, fr);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      // a failed hipMalloc also sets the thread's last error: clear it, or
      // the launch check after the next kernel would report it
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
        return HAPOD_E_NOMEM;
      }
    }
    size_of_[p] = bytes;
    held_ += bytes;
    peak_ = std::max(peak_, held_);
    *out = p;
    return HAPOD_OK;
  }
  void free(void* p) {
    if (!p) return;
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    free_[it->second].push_back(p);
  }
  // give a block back to the device at once instead of caching it
  void free_now(void* p) {
    if (!p) return;
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    held_ -= it->second;
    size_of_.erase(it);
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
  }
  // Return cached blocks until at least `bytes` went back: the smallest
  // block that covers what is still missing, else the largest and repeat.
  // Large blocks are the expensive ones to map again, and the next run of
  // the plan asks for the same sizes.
  void trim_until(size_t bytes) {
    // (cached blocks may still be read by queued work: helpers return them
    // without synchronising their stream)
    (void)hipDeviceSynchronize();
    size_t freed = 0;
    while (freed < bytes) {
      for (auto it = free_.begin(); it != free_.end();)
        it = it->second.empty() ? free_.erase(it) : std::next(it);
      if (free_.empty()) break;
      auto it = free_.lower_bound(bytes - freed);
      if (it == free_.end()) it = std::prev(free_.end());
      void* p = it->second.back();
      it->second.pop_back();
      freed += it->first;
      held_ -= it->first;
      size_of_.erase(p);
      (void)hipFree(p);
      if (verbose_) std::fprintf(stderr, "[hapod pool] return %zu bytes\n", it->first);
    }
  }
  void trim() {
    (void)hipDeviceSynchronize();
    for (auto& kv : free_)
      for (void* p : kv.second) {
        held_ -= size_of_[p];
        size_of_.erase(p);
        (void)hipFree(p);
      }
    free_.clear();
  }
  void release_all() {
    for (auto& kv : size_of_) (void)hipFree(kv.first);
    size_of_.clear();
    free_.clear();
    held_ = 0;
    if (pinned_) (void)hipHostFree(pinned_);
    pinned_ = nullptr;
    pinned_bytes_ = 0;
    if (ring_) (void)hipHostFree(ring_);
    ring_ = nullptr;
    ring_pos_ = 0;
  }
  // A pinned copy of `bytes` host bytes for an upload the caller does not
  // wait for (NULL if no ring could be mapped, or too large): the helpers'
  // descriptor tables go through it, so that they return without a stream
  // synchronisation.  A region is reused only after the ring wraps, which
  // waits for the device to finish everything queued.
  const void* stage(const void* src, size_t bytes) {
    constexpr size_t kRing = size_t(32) << 20;
    const size_t b = align_up(std::max<size_t>(bytes, 1));
    if (b > kRing) return nullptr;
    if (!ring_) {
      if (hipHostMalloc(&ring_, kRing, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ring_ = nullptr;
        return nullptr;
      }
      ring_pos_ = 0;
    }
    if (ring_pos_ + b > kRing) {
      if (hipDeviceSynchronize() != hipSuccess) return nullptr;
      ring_pos_ = 0;
    }
    char* p = (char*)ring_ + ring_pos_;
    std::memcpy(p, src, bytes);
    ring_pos_ += b;
    return p;
  }
  // Pinned host staging of at least `bytes` (grown on demand; its contents
  // do not survive growth).  Small descriptor uploads and readbacks go
  // through it: copies from pageable memory can stall the host for a long
  // and varying time.  The caller orders its uses on one stream.
  char* pinned(size_t bytes) {
    if (bytes <= pinned_bytes_) return (char*)pinned_;
    if (pinned_) (void)hipHostFree(pinned_);
    pinned_ = nullptr;
    pinned_bytes_ = 0;
    const size_t want = std::max<size_t>(align_up(bytes), size_t(64) << 10);
    if (hipHostMalloc(&pinned_, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      pinned_ = nullptr;
      return nullptr;
    }
    pinned_bytes_ = want;
    return (char*)pinned_;
  }
  void set_cap(size_t c) { cap_ = c; }
  size_t held() const { return held_; }
  // the most device memory held since the last reset_peak()
  size_t peak() const { return peak_; }
  void reset_peak() { peak_ = held_; }
  // bytes held in freed blocks, ready for reuse
  size_t cached() const {
    size_t c = 0;
    for (auto& kv : free_) c += kv.first * kv.second.size();
    return c;
  }
  // size of the largest cached block within [lo, hi], 0 if none
  size_t cached_within(size_t lo, size_t hi) const {
    size_t best = 0;
    for (auto it = free_.lower_bound(lo); it != free_.end() && it->first <= hi; ++it)
      if (!it->second.empty()) best = it->first;
    return best;
  }
  // bytes the cap still allows (cached blocks count as available)
  size_t room() const {
    if (!cap_) return SIZE_MAX;
    const size_t used = held_ - cached();
    return cap_ > used ? cap_ - used : 0;
  }

 private:
  std::map<size_t, std::vector<void*>> free_;
  std::map<void*, size_t> size_of_;
  size_t held_ = 0, cap_ = 0, peak_ = 0;
  void* pinned_ = nullptr;
  size_t pinned_bytes_ = 0;
  void* ring_ = nullptr;
  size_t ring_pos_ = 0;
  bool verbose_ = [] {
    const char* v = std::getenv("HAPOD_VERBOSE");
    return v && v[0] == '1';
  }();
};

// Host staging blob that becomes one device blob (descriptor tables).
struct Blob {
  std::vector<char> host;
  size_t add(const void* p, size_t bytes) {
    size_t off = align_up(host.size());
    host.resize(off + bytes);
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <class T> size_t add_vec(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

// ---------------------------------------------------------------------------
// One batch of local PODs (all nodes of a level, or a single node).
// ---------------------------------------------------------------------------
// The dense lift's preconditions on one column table: every column holds
// all n rows, readable to the next multiple of 128 (a plain column only when
// n is a multiple of 128), every column and row block starts 16-byte aligned.
bool dense_cols(int64_t n, int64_t m, const void* const* p, const int64_t* rbs, const int64_t* rows) {
  for (int64_t j = 0; j < m; ++j) {
    if (rows[j] != n || ((uintptr_t)p[j] & 15u) != 0 || (rbs[j] & 1) != 0) return false;
    if (rbs[j] == kRowBlock && n % kRowBlock != 0) return false;
  }
  return true;
}
// ... and on the sizes: m a multiple of 8, the operand's rows whole aligned
// runs of 4 (ldb a multiple of 4, or N a multiple of 128 with ldb even).
bool dense_sizes(int64_t m, int64_t N, int64_t ldb) {
  return m % 8 == 0 && (ldb % 4 == 0 || (N % kLiftTileN == 0 && ldb % 2 == 0));
}

struct PodJob {
  // inputs
  std::vector<const void*> cols;  // host copy of the column pointers
  std::vector<int64_t> rbs;       // row-block stride of every column
  std::vector<int64_t> crows;     // rows every column holds (<= n)
  int64_t n = 0;
  int64_t m = 0;
  double eps = 0.0;
  bool root = false;    // lift with Lambda^{-1/2}
  void* out = nullptr;  // n x m capacity; element (r, c) at out[c * ocs + blk_off(r, obs)]
  // out == nullptr and alloc_rows > 0: the batch allocates the output from the
  // pool once the rank N is known -- alloc_rows x N plain column-major
  // (ocs = alloc_rows, rows past n zero-filled) when plain_out, else n x N
  // row-block tiled (ocs = 128, obs = 128 N)
  int64_t alloc_rows = 0;
  bool plain_out = false;
  int64_t ocs = 0;
  int64_t obs = kRowBlock;
  // outputs (host, after sync)
  int64_t rank = 0;
  std::vector<double> sigma;
  double info[6] = {0, 0, 0, 0, 0, 0};
  int32_t sweeps = 0;
  bool wide = false;
  bool wide_full = false;      // complete tridiagonal reduction: every eigenpair, as Jacobi gives
  bool wide_exhausted = true;  // wide eigensolve reached the Gram's rounding level
  double wide_missing = 0.0;   // energy of unconverged Ritz values above it
  double wide_unresolved = 0.0;  // trace(G) minus the returned eigenvalues
  double wide_slack = 0.0;       // rounding allowance of that difference
  double wide_noise_room = 0.0;  // energy the unresolved eigenvalues may hold
  // block-structured Gram: column ranges [lo, hi) of computed children's
  // scaled modes and sigma^2 of every column (0 outside those ranges)
  std::vector<std::pair<int64_t, int64_t>> sblk;
  std::vector<double> s2;
  bool keep_v = false;      // copy V[:, :N] to a pool block of its own
  // a leaf that may hand its own columns to its parent when its rank is m
  // (host-driven batch: no output, no lift for it then; passed says so)
  bool pass_full = false;
  bool passed = false;
  double* vkeep = nullptr;  // that block (m x N, ld m)
  int64_t cap_hint = 0;     // the node's rank in the plan's previous run (0: none)
};

struct PhaseTimes {
  float gram = 0, eig = 0, trunc = 0, lift = 0;
  float graph = 0;  // batches launched as a hipGraph (phases not separated)
};

// batches of the last run: device-driven (nothing back to the host between
// the Gram and the lift), with the ranks read back before the lift, and
// device-driven ones run again because a rank outgrew its output
struct BatchStats {
  int64_t device = 0, host = 0, reruns = 0;
};

// hipGraphs of device-driven batches (plan option graph_levels), one per
// batch position in a run (level, or wave of leaves): a batch whose
// descriptors, device buffers and launch parameters hash to what the graph
// at its position was captured from replays it; any difference captures
// anew.  Captured on a private stream (default priority), launched on the
// run's stream; the uploads stay outside the graph.
struct GraphCache {
  struct Entry {
    uint64_t sig = 0;
    hipGraphExec_t exec = nullptr;
  };
  bool on = false;
  hipStream_t cap = nullptr;
  std::vector<Entry> entries;
  size_t next = 0;
  int64_t captures = 0, replays = 0;
  ~GraphCache() {
    for (auto& e : entries)
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// FNV-1a over byte ranges
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  }
  template <class T> void val(const T& v) { add(&v, sizeof(v)); }
  template <class T> void vec(const std::vector<T>& v) {
    val(v.size());
    add(v.data(), v.size() * sizeof(T));
  }
};

struct Events {
  hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool ok = false;
  Events() {
    ok = true;
    for (auto& x : e)
      if (hipEventCreate(&x) != hipSuccess) ok = false;
  }
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};


// Tile autotuning.  For a node class of at most 256 columns (compute mode,
// width rounded up to a multiple of 16, height class 2^ceil(log2 n)) seen for
// the first time, the candidate tiles -- the default and its neighbours --
// are timed on a zero buffer of the node's width and up to 2^20 of its rows
// (the kernels' speed does not depend on the values), and the fastest is kept
// for the rest of the process.  Tuning is on when the plan asks for it;
// results are then deterministic for a given tuning table.
constexpr int64_t kTuneMaxCols = 256;
struct TileKey {
  int compute;
  int64_t m;
  int nlog;
  bool operator<(const TileKey& o) const {
    return compute != o.compute ? compute < o.compute : m != o.m ? m < o.m : nlog < o.nlog;
  }
};
std::map<TileKey, int>& tile_table() {
  static std::map<TileKey, int> t;
  return t;
}
std::mutex& tile_mutex() {
  static std::mutex mu;
  return mu;
}
int64_t width_class(int64_t m) { return (m + 15) / 16 * 16; }
int tile_for_node(int compute, int64_t n, int64_t m) {
  int nlog = 0;
  while ((int64_t(1) << nlog) < n && nlog < 62) ++nlog;
  std::lock_guard<std::mutex> lk(tile_mutex());
  auto it = tile_table().find(TileKey{compute, width_class(m), nlog});
  return it != tile_table().end() ? it->second : gram_tile_for(m);
}
hapod_status autotune_tile(int compute, int eb, int64_t n, int64_t m_node, Pool& pool, hipStream_t stream) {
  // wide nodes always take the 128 quad tile: the choice only matters for
  // nodes of a few tiles, whose Gram a short sample represents well
  if (n <= 0 || m_node <= 1 || m_node > kTuneMaxCols) return HAPOD_OK;
  const int64_t m = width_class(m_node);
  int nlog = 0;
  while ((int64_t(1) << nlog) < n && nlog < 62) ++nlog;
  const TileKey key{compute, m, nlog};
  {
    std::lock_guard<std::mutex> lk(tile_mutex());
    if (tile_table().count(key)) return HAPOD_OK;
  }
  const int def = gram_tile_for(m);
  std::vector<int> cand{def};
  if (def > 16) cand.push_back(def / 2);
  if (def < kGramTile) cand.push_back(def * 2);
  // full height up to 2^20 rows and 2 GiB
  const int64_t ns = std::max<int64_t>(
      std::min<int64_t>(std::min<int64_t>(n, int64_t(1) << 20), (int64_t(2) << 30) / (m * eb)) / kRowBlock * kRowBlock,
      std::min<int64_t>(n, kRowBlock));
  void *S = nullptr, *G = nullptr;
  HAPOD_TRY(pool.alloc((size_t)ns * m * eb, &S));
  hapod_status st = pool.alloc(sizeof(double) * m * m, &G);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = def;
  float best_ms = 1e30f;
  if (st == HAPOD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = HAPOD_E_DEVICE;
  if (st == HAPOD_OK) st = launch_zero_bytes(S, (size_t)ns * m * eb, stream);
  for (int t : cand) {
    if (st != HAPOD_OK) break;
    st = gram_impl(compute, eb, ns, m, S, ns, (double*)G, m, stream, t);  // warm-up
    float ms = 0.f;
    if (st == HAPOD_OK && hipEventRecord(e0, stream) != hipSuccess) st = HAPOD_E_DEVICE;
    for (int r = 0; r < 2 && st == HAPOD_OK; ++r) st = gram_impl(compute, eb, ns, m, S, ns, (double*)G, m, stream, t);
    if (st == HAPOD_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = HAPOD_E_DEVICE;
    if (st == HAPOD_OK && ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  pool.free_now(S);
  if (G) pool.free_now(G);
  if (st != HAPOD_OK) return st;
  std::lock_guard<std::mutex> lk(tile_mutex());
  tile_table()[key] = best;
  return HAPOD_OK;
}

// The tile table on disk (autotune_cache): one line per node class,
// "compute width height_log2 tile".  Loaded into the process's table when a
// plan names the file (entries already present win), written back whole
// after every run of a plan with tuning on (to a temporary file first, then
// renamed).
void load_tile_cache(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  std::lock_guard<std::mutex> lk(tile_mutex());
  // line by line: a line that does not parse is skipped, not the rest
  while (std::fgets(line, sizeof(line), f)) {
    int c = 0, nl = 0, t = 0;
    long long w = 0;
    if (std::sscanf(line, "%d %lld %d %d", &c, &w, &nl, &t) == 4 && (t == 16 || t == 32 || t == 64 || t == 128) &&
        c >= 0 && c <= 3 && w > 0 && nl >= 0 && nl <= 62)
      tile_table().emplace(TileKey{c, (int64_t)w, nl}, t);
  }
  std::fclose(f);
}
hapod_status save_tile_cache(const std::string& path) {
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) {
    set_error("autotune_cache: cannot write " + tmp);
    return HAPOD_E_INVALID;
  }
  {
    std::lock_guard<std::mutex> lk(tile_mutex());
    for (const auto& kv : tile_table())
      std::fprintf(f, "%d %lld %d %d\n", kv.first.compute, (long long)kv.first.m, kv.first.nlog, kv.second);
  }
  const bool ok = std::fclose(f) == 0 && std::rename(tmp.c_str(), path.c_str()) == 0;
  if (!ok) {
    set_error("autotune_cache: cannot replace " + path);
    return HAPOD_E_INVALID;
  }
  return HAPOD_OK;
}

// Eigensolver choice.  jacobi_max > 0: Jacobi up to that width, Lanczos
// above.  jacobi_max <= 0 (automatic): Jacobi in LDS up to kAutoJacobiMin;
// between that and kAutoJacobiMax every eigenpair, as Jacobi gives, from a
// Householder reduction to tridiagonal form (one workgroup per node, all
// such nodes of a batch in one launch; 2 ms against Jacobi's 32 ms at 128
// columns); above, Lanczos stopped at the Gram's rounding level.
constexpr int kAutoJacobiMin = 64;
constexpr int kAutoJacobiMax = 256;
constexpr int64_t kLiftTargetItems = 2048;  // lift workgroups per launch to aim for

hapod_status run_pod_batch_impl(hapod_precision prec, std::vector<PodJob>& jobs, int policy_small, int policy_wide,
                                int jacobi_max, Pool& pool, hipStream_t stream, PhaseTimes* times,
                                void** batch_block, bool autotune, bool allow_dev, bool* overflow,
                                BatchStats* bstats, GraphCache* gcache) {
  const int compute = compute_mode(prec);
  const int eb = elem_bytes(prec);
  const int nj = (int)jobs.size();
  if (nj == 0) return HAPOD_OK;
  const double u_p = (prec == HAPOD_FP64) ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
  // the split-BF16 form lifts in split-BF16 too (HAPOD_LIFT_FP32=1: on FP32
  // MFMA, as the FP32 form does)
  static const bool split_lift = [] {
    const char* e = std::getenv("HAPOD_LIFT_FP32");
    return !(e && e[0] == '1');
  }();

  // ---- sizes & scratch layout ---------------------------------------------
  struct Lay {
    size_t cols, rbs, crows, cols2, rbs2, crows2, G, partial, lam, V, B, B32, Bs, sigma, rank, info, jwork, vwork,
        sweeps, hh, hhdiag;
    bool presplit, own256;
    int tile, slots, ntiles, pairs, nchunks;
    int64_t chunk_rows;
  };
  std::vector<Lay> lay(nj);
  size_t total = 0, ttotal = 0;
  int total_pairs = 0;
  const int KB = (compute == 2) ? 32 : 16;
  // enough row chunks to give every CU several workgroups
  int sum_pairs = 0;
  // the Gram compute mode of a node: split-BF16 nodes below the pre-split
  // width run on FP32 MFMA
  auto node_compute = [&](int64_t m) { return (compute == 2 && m < kBf16MinCols) ? 1 : compute; };
  if (autotune)
    for (auto& j : jobs) HAPOD_TRY(autotune_tile(node_compute(j.m), eb, j.n, j.m, pool, stream));
  for (auto& j : jobs) {
    const int tile = tile_for_node(node_compute(j.m), j.n, j.m);
    int nt = (int)((j.m + tile - 1) / tile);
    sum_pairs += nt * (nt + 1) / 2;
  }
  // work items per Gram launch to aim for (row chunks are added until the
  // tile pairs reach it): 8192 measured best on the 2^20 x 8192 star (FP64
  // root Gram 1232 -> 1156 ms against 2048) and the 2^22-row chain (1542 ->
  // 1210 ms); HAPOD_GRAM_ITEMS overrides it
  int item_goal = 8192;
  if (const char* e = std::getenv("HAPOD_GRAM_ITEMS")) {
    const int v = std::atoi(e);
    if (v > 0) item_goal = v;
  }
  const int target_items = std::max(item_goal, sum_pairs);
  // split twins take as much memory as their inputs.  They are made and
  // consumed in groups that fit an arena of at most half of what the device
  // has free (and of what the plan's cap leaves): the Gram of one group runs
  // before the next group's twins overwrite the arena.  A node whose twin
  // alone exceeds the arena splits in registers instead.
  size_t twin_budget = 0;
  if (compute == 2) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      const size_t avail = free_b + pool.cached();
      twin_budget = avail > Pool::kReserve ? (avail - Pool::kReserve) / 2 : 0;
    }
    const size_t room = pool.room();
    if (room / 2 < twin_budget) twin_budget = room / 2;
    // whole GiB: the same level of the next run then asks for the same arena
    // and finds it in the pool's cache
    if (twin_budget >= (size_t(2) << 30)) twin_budget &= ~((size_t(1) << 30) - 1);
    // a cached block near that size (an earlier run's arena) becomes the
    // arena: free memory drifts between runs, and an arena a little larger
    // than every cached block would map memory anew each run
    if (const size_t c = pool.cached_within(twin_budget / 2, twin_budget + twin_budget / 2)) twin_budget = c;
    // HAPOD_TWIN_BUDGET (bytes) lowers the arena further
    if (const char* e = std::getenv("HAPOD_TWIN_BUDGET")) {
      const long long v = std::atoll(e);
      if (v > 0 && (size_t)v < twin_budget) twin_budget = (size_t)v;
    }
  }
  std::vector<int> twin_group(nj, 0);
  std::vector<size_t> twin_off(nj, 0);
  size_t arena_bytes = 0, group_fill = 0;
  int ngroups = 1;
  for (auto& j : jobs) {
    j.wide = (jacobi_max > 0) ? (j.m > jacobi_max) : (j.m > kAutoJacobiMin);
    // a node taken from Jacobi only for speed keeps Jacobi's result: all
    // eigenpairs (a complete tridiagonal reduction) and the same truncation
    // policy
    j.wide_full = j.wide && jacobi_max <= 0 && j.m <= kAutoJacobiMax;
  }
  // Device-driven batch: when every node's eigensolve runs without host
  // steps (Jacobi, or the Householder reduction of a full run), nothing
  // returns to the host between the Gram and the lift: outputs and lift
  // work lists are sized for rank m (the lift's tiles past the rank the
  // truncation writes retire at once) and the ranks come back with the other
  // results at the end.  Not for right-vector runs (their copy of V is sized
  // by the rank); HAPOD_HOST_LEVELS=1 keeps the rank readback.
  static const bool host_levels = [] {
    const char* e = std::getenv("HAPOD_HOST_LEVELS");
    return e && e[0] == '1';
  }();
  bool dev = allow_dev && !host_levels && hh_available();
  // output capacity of a batch-allocated node: its rank in the previous run
  // (the layout of its output then matches a run that read the rank back),
  // else m
  std::vector<int64_t> cap(nj, 0);
  size_t worst_out = 0;
  for (int i = 0; i < nj; ++i) {
    const PodJob& j = jobs[i];
    if (j.keep_v || j.pass_full || (j.m > 0 && j.wide && !(j.wide_full && j.m <= kHouseholderMaxM))) dev = false;
    cap[i] = (j.cap_hint > 0 && j.cap_hint <= j.m) ? j.cap_hint : j.m;
    if (!j.out && j.alloc_rows > 0 && j.m > 0)
      worst_out += align_up(j.plain_out ? (size_t)j.alloc_rows * cap[i] * eb : tiled_bytes(j.n, cap[i], eb));
  }
  // the worst-case outputs must fit a quarter of what the device has free
  // (and of what the plan's cap leaves); else the ranks come back first
  if (dev && worst_out > 0) {
    size_t free_b = 0, total_b = 0;
    size_t room = pool.room();
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      const size_t avail = free_b + pool.cached();
      room = std::min(room, avail > Pool::kReserve ? (avail - Pool::kReserve) / 4 : 0);
    }
    if (worst_out > room) dev = false;
  }
  if (bstats) ++(dev ? bstats->device : bstats->host);
  for (int i = 0; i < nj; ++i) {
    PodJob& j = jobs[i];
    Lay& L = lay[i];
    const int64_t m = j.m;
    L.tile = tile_for_node(node_compute(m), j.n, m);
    // split-BF16: nodes with several column tiles get a split twin of their
    // input once, instead of splitting every element in each tile that reads
    // it; a pre-split twin (every value split once, in a pass of its own)
    // pays when each column block is read by several tiles: above 256
    // columns, or with tiles narrower than 128 (chosen by the tile tuner);
    // below, the 128-column tiles split the FP32 values as they stage them
    L.presplit = (compute == 2 && m >= kBf16MinCols && (L.tile != 128 || m > kStageSplitMaxCols) && j.n > 0 &&
                  tiled_bytes(j.n, m, 4) <= twin_budget);
    // pre-split nodes above 256 columns take 256-column tiles (eight
    // wavefronts of 128 x 64: half the LDS reads per product)
    if (L.presplit && m > kStageSplitMaxCols && L.tile == 128) L.tile = 256;
    // split-BF16 nodes of 129 .. 256 columns: one 256-column tile staged from
    // their own FP32 columns, each value read once (three 128-column tile
    // pairs read every column twice)
    L.own256 = (compute == 2 && !L.presplit && L.tile == 128 && m > 128 && m <= kStageSplitMaxCols);
    if (L.own256) L.tile = 256;
    L.ntiles = (int)((m + L.tile - 1) / L.tile);
    L.pairs = L.ntiles * (L.ntiles + 1) / 2;
    // (sum_pairs counts 128-column pairs: a node on 256-column tiles, whose
    // items carry four times the work, aims at a quarter of the items)
    const int64_t node_items = (int64_t)target_items * L.pairs / std::max(sum_pairs, 1);
    const int per_node_target = std::max(1, (int)node_items);
    L.nchunks = pick_chunks(j.n, L.pairs, per_node_target, 2048);
    int64_t cr = (j.n + L.nchunks - 1) / L.nchunks;
    cr = (cr + kRowBlock - 1) / kRowBlock * kRowBlock;
    if (cr < KB) cr = KB;
    L.chunk_rows = cr;
    L.nchunks = (int)std::max<int64_t>(1, (j.n + cr - 1) / cr);
    auto take = [&](size_t bytes) {
      size_t off = total;
      total = align_up(total + bytes);
      return off;
    };
    // column tables: offsets inside the table region (placed after the rest,
    // filled by one upload)
    auto ttake = [&](size_t bytes) {
      size_t off = ttotal;
      ttotal = align_up(ttotal + bytes);
      return off;
    };
    L.cols = ttake(sizeof(void*) * std::max<int64_t>(m, 1));
    L.rbs = ttake(sizeof(int64_t) * std::max<int64_t>(m, 1));
    L.crows = ttake(sizeof(int64_t) * std::max<int64_t>(m, 1));
    if (L.presplit) {
      const size_t tb = align_up(tiled_bytes(j.n, m, 4));
      if (group_fill + tb > twin_budget) {
        ++ngroups;
        group_fill = 0;
      }
      twin_group[i] = ngroups - 1;
      twin_off[i] = group_fill;
      group_fill += tb;
      arena_bytes = std::max(arena_bytes, group_fill);
    }
    L.cols2 = L.presplit ? ttake(sizeof(void*) * m) : 0;
    L.rbs2 = L.presplit ? ttake(sizeof(int64_t) * m) : 0;
    L.crows2 = L.presplit ? ttake(sizeof(int64_t) * m) : 0;
    L.G = take(sizeof(double) * m * m);
    L.slots = L.nchunks * gram_slots_per_chunk(L.tile);
    L.partial = (L.slots > 1) ? take(sizeof(double) * (size_t)L.pairs * L.slots * L.tile * L.tile) : 0;
    L.lam = take(sizeof(double) * std::max<int64_t>(m, 1));
    L.V = take(sizeof(double) * m * m);
    // lift operand rows padded to a multiple of 4 entries: 16-byte aligned runs
    const int64_t ldb = std::max<int64_t>((m + 3) / 4 * 4, 4);
    L.B = take(sizeof(double) * m * ldb);
    L.B32 = (compute != 0) ? take(sizeof(float) * m * ldb) : 0;
    L.Bs = (compute == 2 && split_lift) ? take(split_operand_bytes(m)) : 0;
    L.sigma = take(sizeof(double) * std::max<int64_t>(m, 1));
    L.rank = take(sizeof(int64_t));
    L.info = take(sizeof(double) * 8);
    L.jwork = (!j.wide && m > kJacobiLdsMax) ? take(sizeof(double) * jacobi_work_doubles((int)m)) : 0;
    L.vwork = (!j.wide) ? take(sizeof(double) * jacobi_vwork_doubles((int)std::max<int64_t>(m, 1))) : 0;
    L.sweeps = take(sizeof(int32_t) * 2);
    // device-driven full runs: the Householder scratch, then trace, sum of
    // eigenvalues and rounding level
    L.hh = (dev && j.wide_full && m > 0) ? take(hh_scratch_bytes(m)) : 0;
    L.hhdiag = (dev && j.wide_full && m > 0) ? take(sizeof(double) * 4) : 0;
    total_pairs += L.pairs;
  }
  const size_t flag_off = total;
  total = align_up(total + 64);
  // the table region goes last
  const size_t tbase = total;
  total += ttotal;
  for (int i = 0; i < nj; ++i) {
    Lay& L = lay[i];
    L.cols += tbase;
    L.rbs += tbase;
    L.crows += tbase;
    if (L.presplit) {
      L.cols2 += tbase;
      L.rbs2 += tbase;
      L.crows2 += tbase;
    }
  }
  char* scratch = nullptr;
  HAPOD_TRY(pool.alloc(total, (void**)&scratch));
  struct Guard {
    Pool& p;
    void* s;
    ~Guard() { p.free(s); }
  } guard{pool, scratch};
  // split-twin arena (released with the batch)
  char* arena = nullptr;
  if (arena_bytes > 0) HAPOD_TRY(pool.alloc(arena_bytes, (void**)&arena));
  struct GuardA {
    Pool& p;
    void* s;
    ~GuardA() { p.free(s); }
  } guarda{pool, arena};
  std::vector<void*> split_buf(nj, nullptr);
  std::vector<std::vector<const void*>> cols2(nj);
  std::vector<std::vector<int64_t>> rbs2(nj), crows2(nj);
  for (int i = 0; i < nj; ++i) {
    if (!lay[i].presplit) continue;
    const int64_t m = jobs[i].m;
    split_buf[i] = arena + twin_off[i];
    cols2[i] = tiled_table(split_buf[i], m, 4);
    rbs2[i].assign((size_t)m, tiled_rbs(m));
    crows2[i].assign((size_t)m, jobs[i].n);
  }

  // ---- descriptor tables ----------------------------------------------------
  std::vector<GramNode> gnodes(nj);
  std::vector<GramItem> gitems;
  // per twin group: (default compute, FP32) x (tile 128, 64, 32, 16) x (scalar,
  // vector runs), slot 16: split-BF16 128-column tiles staged through LDS,
  // slot 17: pre-split 256-column tiles, slot 18: 256-column tiles staged
  // from FP32 columns
  std::vector<std::array<std::vector<GramItem>, 19>> items_by_tile(ngroups);
  auto tile_slot = [](int t) { return t == 128 ? 0 : t == 64 ? 1 : t == 32 ? 2 : 3; };
  int max_reduce_tile = 0;
  std::vector<int32_t> rpairs, rnode;
  std::vector<GramFill> fills;
  std::vector<double> s2_all;
  std::vector<EigNode> enodes_small, enodes_big;
  std::vector<TruncNode> tnodes(nj);

  int pair_base = 0, max_small = 0, max_big = 0;
  for (int i = 0; i < nj; ++i) {
    PodJob& j = jobs[i];
    Lay& L = lay[i];
    const int64_t m = j.m;
    // vector runs need 16-byte aligned columns (the split twin always is)
    bool vec = (L.chunk_rows % KB) == 0;
    if (!L.presplit)
      for (const void* c : j.cols)
        if (((uintptr_t)c & 15u) != 0) vec = false;
    GramNode& g = gnodes[i];
    g.cols = (const void* const*)(scratch + (L.presplit ? L.cols2 : L.cols));
    g.rbs = (const int64_t*)(scratch + (L.presplit ? L.rbs2 : L.rbs));
    g.crows = (const int64_t*)(scratch + (L.presplit ? L.crows2 : L.crows));
    g.split = L.presplit ? 1 : 0;
    g.n = j.n;
    g.chunk_rows = L.chunk_rows;
    g.G = (double*)(scratch + L.G);
    g.partial = L.slots > 1 ? (double*)(scratch + L.partial) : nullptr;
    g.ldg = m;
    g.m = (int32_t)m;
    g.nchunks = L.nchunks;
    g.ntiles = L.ntiles;
    g.pair_base = pair_base;
    g.tile = L.tile;
    // split-BF16 nodes narrower than the pre-split threshold run their Gram on
    // FP32 MFMA: splitting in registers costs more VALU time than the three
    // BF16 products save at these widths (launch slots of their own)
    const bool f32 = (node_compute(m) != compute);
    const bool staged = !f32 && compute == 2 && L.tile == 128;
    std::vector<GramItem>& gi =
        items_by_tile[twin_group[i]][L.tile == 256 ? (L.own256 ? 18 : 17)
                                     : staged ? 16 : (f32 ? 8 : 0) + 2 * tile_slot(L.tile) + (vec ? 1 : 0)];
    // Item order.  The workgroups an XCD runs at once take consecutive items
    // (see xcd_item), so consecutive items should share column blocks: for
    // each row chunk, the tile pairs go in super-tiles of kSuperI x kSuperJ
    // pairs, whose concurrent workgroups read kSuperI + kSuperJ column blocks
    // of a row stripe instead of about one block per workgroup.  Pair indices
    // stay row-major over the upper triangle (partial slots, reduction).
    const int nt = L.ntiles;
    auto pair_of = [nt](int ti, int tj) { return ti * nt - ti * (ti - 1) / 2 + (tj - ti); };
    // block-structured Gram: a tile wholly inside one computed child's
    // columns carries that child's id; pairs of tiles of one child are set
    // to diag(sigma^2) instead of computed (Def. 3.2: the child's inputs to
    // this node are its scaled orthonormal modes)
    std::vector<int> tile_blk(nt, -1);
    for (size_t q = 0; q < j.sblk.size(); ++q)
      for (int ti = 0; ti < nt; ++ti) {
        const int64_t lo = (int64_t)ti * L.tile, hi = std::min<int64_t>(m, lo + L.tile);
        if (lo >= j.sblk[q].first && hi <= j.sblk[q].second) tile_blk[ti] = (int)q;
      }
    auto set_pair = [&](int ti, int tj) { return tile_blk[ti] >= 0 && tile_blk[ti] == tile_blk[tj]; };
    // the rows a tile holds: the most of its columns' (inputs of uneven height
    // leave whole row chunks zero for some tile pairs)
    std::vector<int64_t> tile_rows(nt, 0);
    for (int64_t c = 0; c < m; ++c) {
      int64_t& tr = tile_rows[c / L.tile];
      tr = std::max(tr, j.crows[(size_t)c]);
    }
    for (int c = 0; c < L.nchunks; ++c)
      for (int I = 0; I < nt; I += kSuperI)
        for (int J = (I / kSuperJ) * kSuperJ; J < nt; J += kSuperJ)
          for (int ti = I; ti < std::min(I + kSuperI, nt); ++ti)
            for (int tj = std::max(J, ti); tj < std::min(J + kSuperJ, nt); ++tj)
              if (!set_pair(ti, tj))
                gi.push_back(GramItem{i, (int16_t)ti, (int16_t)tj, c, pair_base + pair_of(ti, tj),
                                      std::min(tile_rows[ti], tile_rows[tj])});
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = ti; tj < nt; ++tj) {
        if (set_pair(ti, tj)) {
          const int r0 = ti * L.tile, c0 = tj * L.tile;
          fills.push_back(GramFill{g.G, m, (int64_t)s2_all.size(), r0, c0, (int)std::min<int64_t>(L.tile, m - r0),
                                   (int)std::min<int64_t>(L.tile, m - c0)});
        } else if (L.slots > 1) {
          rpairs.push_back(pair_base + pair_of(ti, tj));
          rnode.push_back(i);
          max_reduce_tile = std::max(max_reduce_tile, L.tile);
        }
      }
    if (!j.s2.empty()) s2_all.insert(s2_all.end(), j.s2.begin(), j.s2.end());
    pair_base += L.pairs;
    if (!j.wide && m > 0) {
      EigNode e{};
      e.G = g.G;
      e.work = L.jwork ? (double*)(scratch + L.jwork) : nullptr;
      e.Vwork = (double*)(scratch + L.vwork);
      e.lambda = (double*)(scratch + L.lam);
      e.V = (double*)(scratch + L.V);
      e.ldg = m;
      e.ldv = m;
      e.m = (int32_t)m;
      e.sweeps = (int32_t*)(scratch + L.sweeps);
      if (m <= kJacobiLdsMax) {
        enodes_small.push_back(e);
        max_small = std::max<int>(max_small, (int)m);
      } else {
        enodes_big.push_back(e);
        max_big = std::max<int>(max_big, (int)m);
      }
    }
    TruncNode& t = tnodes[i];
    t.lambda = (double*)(scratch + L.lam);
    t.V = (double*)(scratch + L.V);
    t.B = (double*)(scratch + L.B);
    t.B32 = (compute != 0) ? (float*)(scratch + L.B32) : nullptr;
    t.sigma = (double*)(scratch + L.sigma);
    t.rank = (int64_t*)(scratch + L.rank);
    t.info = (double*)(scratch + L.info);
    t.eps2 = j.eps * j.eps;
    t.floor_abs = 0.0;
    t.ldv = m;
    t.ldb = std::max<int64_t>((m + 3) / 4 * 4, 4);
    t.m = (int32_t)m;
    t.policy = (j.wide && !j.wide_full) ? policy_wide : policy_small;
    t.root = j.root ? 1 : 0;
  }

  Blob blob;
  // the column tables of every node, as one image of the table region
  std::vector<char> timg(ttotal);
  auto put = [&](size_t abs_off, const void* p, size_t bytes) {
    if (bytes) std::memcpy(timg.data() + (abs_off - tbase), p, bytes);
  };
  for (int i = 0; i < nj; ++i) {
    const size_t m = (size_t)jobs[i].m;
    if (m == 0) continue;
    put(lay[i].cols, jobs[i].cols.data(), sizeof(void*) * m);
    put(lay[i].rbs, jobs[i].rbs.data(), sizeof(int64_t) * m);
    put(lay[i].crows, jobs[i].crows.data(), sizeof(int64_t) * m);
    if (lay[i].presplit) {
      put(lay[i].cols2, cols2[i].data(), sizeof(void*) * m);
      put(lay[i].rbs2, rbs2[i].data(), sizeof(int64_t) * m);
      put(lay[i].crows2, crows2[i].data(), sizeof(int64_t) * m);
    }
  }
  // Launches whose nodes each have one tile pair (no column blocks to share
  // in L2, so the super-tile order does not matter): nodes of very different
  // heights give items of very different lengths.  Largest first on every
  // XCD: xcd_item hands XCD x a contiguous range of the launch's items, so
  // the k-th largest item goes to XCD k % 8, position k / 8 of its range.
  for (int gr = 0; gr < ngroups; ++gr)
  for (int slot = 0; slot < 19; ++slot) {
    auto& v = items_by_tile[gr][slot];
    const size_t N = v.size();
    if (N < 16) continue;
    bool single = true;
    for (const GramItem& it : v) single = single && lay[it.node].pairs == 1;
    if (!single) continue;
    auto rows = [&](const GramItem& it) {
      const Lay& L = lay[it.node];
      const int64_t r0 = (int64_t)it.chunk * L.chunk_rows;
      const int64_t r1 = std::min(std::min<int64_t>(jobs[it.node].n, r0 + L.chunk_rows), it.rlim);
      return std::max<int64_t>(0, r1 - r0);
    };
    std::vector<GramItem> by_rows(v);
    std::stable_sort(by_rows.begin(), by_rows.end(),
                     [&](const GramItem& a, const GramItem& b) { return rows(a) > rows(b); });
    const size_t q = N / 8, r = N % 8;
    for (size_t k = 0; k < N; ++k) {
      const size_t x = k % 8, pos = k / 8;
      const size_t start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
      v[start + pos] = by_rows[k];
    }
  }
  std::vector<std::vector<GramLaunch>> glaunch(ngroups);
  for (int gr = 0; gr < ngroups; ++gr)
    for (int t = 0; t < 19; ++t) {
      const auto& v = items_by_tile[gr][t];
      if (v.empty()) continue;
      if (t >= 16)
        glaunch[gr].push_back(GramLaunch{t == 16 ? 128 : 256, t == 18 ? 3 : 2, (int32_t)gitems.size(),
                                         (int32_t)v.size(), -1});
      else
        glaunch[gr].push_back(GramLaunch{128 >> ((t & 7) / 2), t & 1, (int32_t)gitems.size(), (int32_t)v.size(),
                                         t >= 8 ? 1 : -1});
      gitems.insert(gitems.end(), v.begin(), v.end());
    }
  // device-driven full runs: descriptors of the Householder eigensolve and
  // of its back-transformation; the truncation reads their rounding level
  std::vector<char> hh_img;
  std::vector<LiftNode> hh_lift;
  std::vector<int> hh_idx;
  int64_t hh_mmax = 0;
  int hh_items = 0;
  if (dev)
    for (int i = 0; i < nj; ++i) {
      if (!jobs[i].wide_full || jobs[i].m <= 0) continue;
      const int64_t m = jobs[i].m;
      const size_t nb = hh_node_bytes();
      hh_img.resize(hh_img.size() + nb);
      double* diag = (double*)(scratch + lay[i].hhdiag);
      LiftNode l{};
      hh_describe(m, gnodes[i].G, m, (double*)(scratch + lay[i].lam), (double*)(scratch + lay[i].V), m,
                  scratch + lay[i].hh, u_p, diag + 2, diag, hh_img.data() + hh_idx.size() * nb, &l);
      l.item_base = hh_items;
      hh_items += l.row_tiles * l.col_tiles;
      hh_lift.push_back(l);
      hh_idx.push_back(i);
      hh_mmax = std::max(hh_mmax, m);
      tnodes[i].floor_ptr = diag + 2;
    }
  // outputs sized by the ranks (worst case m in a device-driven batch),
  // carved from one block for the batch (one allocation instead of one per
  // node; the caller frees the block once every node in it has been
  // consumed), and the lift work lists: nodes of rank <= 64 take the narrow
  // lift (256 x 64 tiles), the others 128 x 128 tiles, each kind one launch
  std::vector<LiftNode> lnodes[2];
  int lift_items[2] = {0, 0};
  char* out_block_mine = nullptr;
  auto build_lifts = [&](const std::vector<int64_t>& ranks, bool worst) -> hapod_status {
    std::vector<size_t> out_off(nj, 0);
    size_t out_total = 0;
    for (int i = 0; i < nj; ++i) {
      const PodJob& j = jobs[i];
      if (j.out || j.alloc_rows <= 0 || j.m <= 0 || ranks[i] <= 0) continue;
      out_off[i] = out_total;
      out_total = align_up(out_total + (j.plain_out ? (size_t)j.alloc_rows * ranks[i] * eb
                                                    : tiled_bytes(j.n, ranks[i], eb)));
    }
    char* out_block = nullptr;
    if (out_total > 0) {
      HAPOD_TRY(pool.alloc(out_total, (void**)&out_block));
      out_block_mine = out_block;
      if (batch_block) *batch_block = out_block;
    }
    for (int i = 0; i < nj; ++i) {
      PodJob& j = jobs[i];
      if (j.out || j.alloc_rows <= 0 || j.m <= 0 || ranks[i] <= 0) continue;
      const int64_t N = ranks[i];
      const size_t bytes = j.plain_out ? (size_t)j.alloc_rows * N * eb : tiled_bytes(j.n, N, eb);
      j.out = out_block + out_off[i];
      if (j.plain_out) {
        j.ocs = j.alloc_rows;
        j.obs = kRowBlock;
        if (j.n < j.alloc_rows) HAPOD_TRY(launch_zero_bytes(j.out, bytes, stream));
      } else {
        j.ocs = kRowBlock;
        j.obs = tiled_rbs(N);
      }
    }
    // several row tiles per workgroup when there are many: the column table
    // and the node lookup are then paid once per group of tiles (sized for
    // one column tile per node when the ranks are worst cases: the items of
    // column tiles past the rank retire at once and must not thin out the
    // rest)
    int64_t lift_tiles = 0;
    for (int i = 0; i < nj; ++i)
      if (jobs[i].m > 0 && jobs[i].n > 0 && ranks[i] > 0) {
        const bool nar = ranks[i] <= kLiftTileN / 2;
        const int64_t tm = nar ? kLiftNarrowM : kLiftTileM, tn = nar ? kLiftTileN / 2 : kLiftTileN;
        lift_tiles += ((jobs[i].n + tm - 1) / tm) * (worst ? 1 : (ranks[i] + tn - 1) / tn);
      }
    const int rt_per = (int)std::max<int64_t>(1, std::min<int64_t>(16, lift_tiles / kLiftTargetItems));
    for (int i = 0; i < nj; ++i) {
      const PodJob& j = jobs[i];
      if (j.m <= 0 || j.n <= 0 || ranks[i] <= 0) continue;
      const int nar = ranks[i] <= kLiftTileN / 2 ? 1 : 0;
      const int64_t tm = nar ? kLiftNarrowM : kLiftTileM, tn = nar ? kLiftTileN / 2 : kLiftTileN;
      LiftNode l{};
      l.cols = (const void* const*)(scratch + lay[i].cols);
      l.rbs = (const int64_t*)(scratch + lay[i].rbs);
      l.crows = (const int64_t*)(scratch + lay[i].crows);
      l.B = tnodes[i].B;
      l.B32 = tnodes[i].B32;
      l.Bs = lay[i].Bs ? (char*)(scratch + lay[i].Bs) : nullptr;
      l.rank = tnodes[i].rank;
      l.out = j.out;
      l.n = j.n;
      l.ldb = tnodes[i].ldb;
      l.ocs = j.ocs;
      l.obs = j.obs;
      l.m = (int32_t)j.m;
      l.row_tiles = (int32_t)((j.n + tm - 1) / tm);
      l.col_tiles = (int32_t)((ranks[i] + tn - 1) / tn);
      l.item_base = lift_items[nar];
      l.rt_per = rt_per;
      lift_items[nar] += ((l.row_tiles + rt_per - 1) / rt_per) * l.col_tiles;
      lnodes[nar].push_back(l);
    }
    return HAPOD_OK;
  };
  // (caller-provided outputs hold m columns: capacity m, no cap)
  std::vector<char> capped(nj, 0);
  if (dev) {
    std::vector<int64_t> worst(nj);
    for (int i = 0; i < nj; ++i) {
      capped[i] = !jobs[i].out && jobs[i].alloc_rows > 0;
      worst[i] = capped[i] ? cap[i] : jobs[i].m;
    }
    HAPOD_TRY(build_lifts(worst, true));
    for (int k = 0; k < 2; ++k)
      for (LiftNode& l : lnodes[k]) {
        int i = 0;
        while (i < nj && tnodes[i].rank != l.rank) ++i;
        if (i < nj && capped[i]) l.ncap = cap[i];
      }
  }
  std::vector<LiftNode> lall(lnodes[0]);
  lall.insert(lall.end(), lnodes[1].begin(), lnodes[1].end());
  const size_t o_g = blob.add_vec(gnodes), o_gi = blob.add_vec(gitems), o_rp = blob.add_vec(rpairs),
               o_rn = blob.add_vec(rnode), o_es = blob.add_vec(enodes_small), o_eb = blob.add_vec(enodes_big),
               o_t = blob.add_vec(tnodes), o_fill = blob.add_vec(fills), o_s2 = blob.add_vec(s2_all),
               o_hh = blob.add_vec(hh_img), o_hhl = blob.add_vec(hh_lift), o_l = blob.add_vec(lall);
  char* dblob = nullptr;
  HAPOD_TRY(pool.alloc(blob.host.size(), (void**)&dblob));
  struct Guard2 {
    Pool& p;
    void* s;
    ~Guard2() { p.free(s); }
  } guard2{pool, dblob};
  HAPOD_HIP(hipMemcpyAsync(dblob, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, stream));
  if (ttotal > 0)
    HAPOD_HIP(hipMemcpyAsync(scratch + tbase, timg.data(), ttotal, hipMemcpyHostToDevice, stream));
  int32_t* d_flag = (int32_t*)(scratch + flag_off);
  // the split-BF16 form lifts with three BF16 products per term: a lift of
  // N output columns does 2 N flops per 4 input bytes, above the FP32 MFMA
  // peak's share of HBM bandwidth once N passes about 40, while the BF16
  // products keep it bandwidth-bound (the operand is split once, below)
  const int lift_compute = (compute == 2 && !split_lift) ? 1 : compute;
  // FP64: the 128 x 128 lift takes the unguarded loads when every node's
  // columns and sizes allow them
  bool lift_dense = (lift_compute == 0);
  for (int i = 0; i < nj && lift_dense; ++i) {
    const PodJob& j = jobs[i];
    if (j.m <= 0 || j.n <= 0) continue;
    lift_dense = dense_sizes(j.m, j.m, tnodes[i].ldb) && (((uintptr_t)tnodes[i].B & 15u) == 0) &&
                 dense_cols(j.n, j.m, j.cols.data(), j.rbs.data(), j.crows.data());
  }
  // ---- a device-driven batch as a hipGraph: replay the one captured at this
  // position when everything the launches read hashes the same, else capture
  GraphCache* gc = (dev && gcache && gcache->on) ? gcache : nullptr;
  GraphCache::Entry* ge = nullptr;
  bool replay = false, capturing = false;
  hipStream_t ls = stream;  // the stream the launches below go to
  uint64_t sig = 0;
  if (gc) {
    Fnv f;
    f.vec(blob.host);
    f.vec(timg);
    f.val(scratch);
    f.val(dblob);
    f.val(arena);
    f.val(tbase);
    f.val(compute);
    f.val(lift_compute);
    f.val(ngroups);
    for (const auto& v : glaunch) f.vec(v);
    for (void* b : split_buf) f.val(b);
    for (const auto& L : lay) f.val(L);
    for (const auto& j : jobs) {
      f.val(j.n);
      f.val(j.m);
    }
    f.val(rpairs.size());
    f.val(max_reduce_tile);
    f.val(fills.size());
    f.val(enodes_small.size());
    f.val(enodes_big.size());
    f.val(max_small);
    f.val(max_big);
    f.val(hh_idx.size());
    f.val(hh_mmax);
    f.val(hh_items);
    f.val(lift_items);
    sig = f.h;
    const size_t k = gc->next++;
    if (gc->entries.size() <= k) gc->entries.resize(k + 1);
    ge = &gc->entries[k];
    if (ge->exec && ge->sig == sig) {
      replay = true;
    } else {
      if (ge->exec) {
        HAPOD_HIP(hipGraphExecDestroy(ge->exec));
        ge->exec = nullptr;
      }
      if (!gc->cap) HAPOD_HIP(hipStreamCreateWithFlags(&gc->cap, hipStreamNonBlocking));
      HAPOD_HIP(hipStreamBeginCapture(gc->cap, hipStreamCaptureModeRelaxed));
      ls = gc->cap;
      capturing = true;
    }
  }
  // a capture left open by an early return is ended (and dropped) here
  struct CaptureGuard {
    hipStream_t s;
    bool* on;
    ~CaptureGuard() {
      if (*on) {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      }
    }
  } cap_guard{ls, &capturing};
  // the host-mode lift descriptors, freed after the final synchronisation
  char* lift_desc_owned = nullptr;
  struct Guard3 {
    Pool& p;
    char*& s;
    ~Guard3() {
      if (s) p.free(s);
    }
  } guard3{pool, lift_desc_owned};
  Events ev;
  const bool tev = times && ev.ok && !gc;  // phase events (not inside a graph)
  if (times && ev.ok && gc) HAPOD_HIP(hipEventRecord(ev.e[0], stream));
  if (!replay) {
    HAPOD_TRY(launch_zero_bytes(d_flag, 64, ls));

    if (tev) HAPOD_HIP(hipEventRecord(ev.e[0], stream));
    // ---- split twins, then Gram, one twin group at a time; then the reduction
    for (int gr = 0; gr < ngroups; ++gr) {
      for (int i = 0; i < nj; ++i)
        if (lay[i].presplit && twin_group[i] == gr)
          HAPOD_TRY(launch_split_cols(jobs[i].n, jobs[i].m, (const void* const*)(scratch + lay[i].cols),
                                      (const int64_t*)(scratch + lay[i].rbs),
                                      (const int64_t*)(scratch + lay[i].crows), (float*)split_buf[i], ls));
      HAPOD_TRY(launch_gram(compute, (const GramNode*)(dblob + o_g), (const GramItem*)(dblob + o_gi),
                            glaunch[gr].data(), (int)glaunch[gr].size(), nullptr, nullptr, 0, 0, ls));
    }
    HAPOD_TRY(launch_gram(compute, (const GramNode*)(dblob + o_g), (const GramItem*)(dblob + o_gi), nullptr, 0,
                          (const int32_t*)(dblob + o_rp), (const int32_t*)(dblob + o_rn), (int)rpairs.size(),
                          max_reduce_tile, ls));
    HAPOD_TRY(launch_gram_fill((const GramFill*)(dblob + o_fill), (int)fills.size(), (const double*)(dblob + o_s2),
                               ls));
    for (int i = 0; i < nj; ++i) HAPOD_TRY(launch_check_diag(gnodes[i].G, gnodes[i].ldg, jobs[i].m, d_flag, ls));
    if (tev) HAPOD_HIP(hipEventRecord(ev.e[1], stream));
    // ---- eigensolve -----------------------------------------------------------
    if (!enodes_small.empty())
      HAPOD_TRY(launch_jacobi((const EigNode*)(dblob + o_es), (int)enodes_small.size(), max_small, ls));
    if (!enodes_big.empty())
      HAPOD_TRY(launch_jacobi((const EigNode*)(dblob + o_eb), (int)enodes_big.size(), max_big, ls));
    // wide nodes: one batched Krylov eigensolve for all of them (device-driven
    // batch: the Householder full runs, launched with no host step)
    std::vector<WideResult> wres(nj);
    if (dev) {
      HAPOD_TRY(hh_launch(dblob + o_hh, (int)hh_idx.size(), hh_mmax, (const LiftNode*)(dblob + o_hhl), hh_items,
                          ls));
    } else {
      std::vector<WideJob> wj;
      for (int i = 0; i < nj; ++i) {
        if (!jobs[i].wide || jobs[i].m <= 0) continue;
        wj.push_back(WideJob{gnodes[i].G, jobs[i].m, jobs[i].m, (double*)(scratch + lay[i].lam),
                             (double*)(scratch + lay[i].V), jobs[i].m, jobs[i].wide_full, &wres[i]});
      }
      if (!wj.empty()) HAPOD_TRY(wide_eigh_batch(wj, u_p, &pool_alloc_cb, &pool_free_cb, &pool, ls));
    }
    for (int i = 0; i < nj; ++i) {
      if (dev || !jobs[i].wide || jobs[i].m <= 0) continue;
      const WideResult& wr = wres[i];
      // eigenvalues beyond the computed block are set to zero by wide_eigh;
      // the floor of the truncation is the Gram's rounding level
      tnodes[i].floor_abs = wr.floor_abs;
      jobs[i].sweeps = wr.iterations;
      jobs[i].wide_exhausted = wr.exhausted;
      jobs[i].wide_missing = wr.missing;
      jobs[i].wide_unresolved = wr.unresolved;
      // the difference trace - sum(theta) carries the rounding of every
      // eigenvalue and of the diagonal: allow 16 (block + sqrt(m)) u_p |trace|
      jobs[i].wide_slack = 16.0 * (wr.block + std::sqrt((double)jobs[i].m)) * u_p * std::fabs(wr.trace);
      // the eigenvalues past the block lie below the resolved level: up to
      // (m - block) noise of unresolved energy is consistent with that (the
      // truncation then cannot certify eps below the noise, as for any Gram of
      // this precision); more means a large eigenvalue was never seen
      jobs[i].wide_noise_room = (double)(jobs[i].m - wr.block) * wr.noise;
      // the energy of the eigenvalues not returned (beyond the rounding
      // allowance) is discarded whatever the rank: the truncation gets the
      // rest of the budget (Def. 2.5 counts every discarded direction)
      tnodes[i].eps2 = std::max(0.0, jobs[i].eps * jobs[i].eps - std::max(0.0, wr.unresolved - jobs[i].wide_slack));
      if (jobs[i].wide_full && wr.unresolved > jobs[i].wide_slack) {
        // the Krylov space broke down before spanning the matrix (an exact
        // multiplicity): fall back to the dense Jacobi eigensolver
        const int m = (int)jobs[i].m;
        if (const char* v = std::getenv("HAPOD_VERBOSE"))
          if (v[0] == '1')
            std::fprintf(stderr, "[hapod] m=%d: Krylov run left %.3e of trace %.3e unresolved (slack %.3e): Jacobi\n",
                         m, wr.unresolved, wr.trace, jobs[i].wide_slack);
        void *jw = nullptr, *vw = nullptr, *de = nullptr;
        HAPOD_TRY(pool.alloc(sizeof(double) * jacobi_work_doubles(m), &jw));
        hapod_status s = pool.alloc(sizeof(double) * jacobi_vwork_doubles(m), &vw);
        if (s == HAPOD_OK) s = pool.alloc(sizeof(EigNode), &de);
        if (s == HAPOD_OK) {
          EigNode e{};
          e.G = gnodes[i].G;
          e.work = (double*)jw;
          e.Vwork = (double*)vw;
          e.lambda = (double*)(scratch + lay[i].lam);
          e.V = (double*)(scratch + lay[i].V);
          e.ldg = m;
          e.ldv = m;
          e.m = m;
          s = hipMemcpyAsync(de, &e, sizeof(e), hipMemcpyHostToDevice, ls) == hipSuccess ? HAPOD_OK : HAPOD_E_DEVICE;
          if (s == HAPOD_OK) s = launch_jacobi((const EigNode*)de, 1, m, ls);
          if (s == HAPOD_OK && hipStreamSynchronize(ls) != hipSuccess) s = HAPOD_E_DEVICE;
        }
        if (de) pool.free(de);
        if (vw) pool.free(vw);
        pool.free(jw);
        if (s != HAPOD_OK) return s;
        jobs[i].wide_unresolved = 0.0;
        jobs[i].wide_missing = 0.0;
        jobs[i].wide_noise_room = 0.0;
        jobs[i].wide_exhausted = true;
        tnodes[i].eps2 = jobs[i].eps * jobs[i].eps;
      }
    }
    if (tev) HAPOD_HIP(hipEventRecord(ev.e[2], stream));
    // wide nodes changed floor_abs on the host: refresh the descriptors (one
    // copy through pinned staging)
    bool any_wide = false;
    for (int i = 0; i < nj; ++i) any_wide |= jobs[i].wide && !dev;
    char* pin = dev ? nullptr : pool.pinned(std::max(sizeof(TruncNode), sizeof(int64_t)) * (size_t)nj);
    if (!dev && !pin) {
      set_error("hipHostMalloc of the descriptor staging failed");
      return HAPOD_E_NOMEM;
    }
    if (any_wide) {
      std::memcpy(pin, tnodes.data(), sizeof(TruncNode) * nj);
      HAPOD_HIP(hipMemcpyAsync(dblob + o_t, pin, sizeof(TruncNode) * nj, hipMemcpyHostToDevice, ls));
    }
    // ---- truncation -----------------------------------------------------------
    HAPOD_TRY(launch_truncate((const TruncNode*)(dblob + o_t), nj, ls));
    if (tev) HAPOD_HIP(hipEventRecord(ev.e[3], stream));
    // ---- lift, sized by the ranks just computed (device-driven batch: by the
    // worst case, built before the launches) ----------------------------------
    // (the ranks come back through the same staging: stream order puts these
    // copies after the descriptor upload that read it)
    char* dlift = nullptr;
    bool dlift_owned = false;
    if (dev) {
      dlift = dblob + o_l;
    } else {
      std::vector<int64_t> ranks(nj, 0);
      for (int i = 0; i < nj; ++i)
        HAPOD_HIP(hipMemcpyAsync(pin + i * sizeof(int64_t), scratch + lay[i].rank, sizeof(int64_t),
                                 hipMemcpyDeviceToHost, ls));
      HAPOD_HIP(hipStreamSynchronize(ls));
      std::memcpy(ranks.data(), pin, sizeof(int64_t) * nj);
      // right singular vectors kept for the factorisation of the snapshot map:
      // the first N eigenvectors (columns of V, ld m) are contiguous
      for (int i = 0; i < nj; ++i) {
        PodJob& j = jobs[i];
        if (!j.keep_v || ranks[i] <= 0 || j.m <= 0) continue;
        const size_t bytes = sizeof(double) * (size_t)j.m * ranks[i];
        HAPOD_TRY(pool.alloc(bytes, (void**)&j.vkeep));
        HAPOD_HIP(hipMemcpyAsync(j.vkeep, scratch + lay[i].V, bytes, hipMemcpyDeviceToDevice, ls));
      }
      // a full-rank leaf that may pass its columns on gets no output and no lift
      std::vector<int64_t> lranks(ranks);
      for (int i = 0; i < nj; ++i) {
        PodJob& j = jobs[i];
        j.passed = j.pass_full && !j.out && j.m > 0 && ranks[i] == j.m;
        if (j.passed) lranks[i] = 0;
      }
      HAPOD_TRY(build_lifts(lranks, false));
      if (!lnodes[0].empty() || !lnodes[1].empty()) {
        std::vector<LiftNode> all(lnodes[0]);
        all.insert(all.end(), lnodes[1].begin(), lnodes[1].end());
        HAPOD_TRY(pool.alloc(sizeof(LiftNode) * all.size(), (void**)&dlift));
        dlift_owned = true;
        HAPOD_HIP(hipMemcpy(dlift, all.data(), sizeof(LiftNode) * all.size(), hipMemcpyHostToDevice));
      }
    }
    const size_t nl0 = lnodes[0].size(), nl1 = lnodes[1].size();
    lift_desc_owned = dlift_owned ? dlift : nullptr;
    if (tev) HAPOD_HIP(hipEventRecord(ev.e[3], stream));
    if (lift_compute == 2 && nl0 + nl1 > 0) {
      int64_t max_m = 0;
      for (int i = 0; i < nj; ++i) max_m = std::max(max_m, jobs[i].m);
      HAPOD_TRY(launch_split_operand((const LiftNode*)dlift, (int)(nl0 + nl1), max_m, ls));
    }
    if (nl0 && lift_dense)
      HAPOD_TRY(launch_lift_dense((const LiftNode*)dlift, (int)nl0, lift_items[0], ls));
    else if (nl0)
      HAPOD_TRY(launch_lift(lift_compute, (const LiftNode*)dlift, (int)nl0, lift_items[0], ls, false));
    if (nl1)
      HAPOD_TRY(launch_lift(lift_compute, (const LiftNode*)dlift + nl0, (int)nl1, lift_items[1], ls, true));
    if (tev) HAPOD_HIP(hipEventRecord(ev.e[4], stream));

  }
  if (capturing) {
    hipGraph_t g = nullptr;
    capturing = false;
    HAPOD_HIP(hipStreamEndCapture(gc->cap, &g));
    const hipError_t ie = hipGraphInstantiate(&ge->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      ge->exec = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      return HAPOD_E_DEVICE;
    }
    ge->sig = sig;
    ++gc->captures;
  } else if (replay) {
    ++gc->replays;
  }
  if (gc) {
    HAPOD_HIP(hipGraphLaunch(ge->exec, stream));
    if (times && ev.ok) HAPOD_HIP(hipEventRecord(ev.e[4], stream));
  }

  // ---- results ----------------------------------------------------------------
  HAPOD_HIP(hipStreamSynchronize(stream));
  int32_t flag = 0;
  HAPOD_HIP(hipMemcpy(&flag, d_flag, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) {
    set_error("non-finite Gram diagonal: the input holds NaN or Inf");
    return HAPOD_E_NUMERIC;
  }
  for (int i = 0; i < nj; ++i) {
    PodJob& j = jobs[i];
    HAPOD_HIP(hipMemcpy(&j.rank, scratch + lay[i].rank, sizeof(int64_t), hipMemcpyDeviceToHost));
    HAPOD_HIP(hipMemcpy(j.info, scratch + lay[i].info, sizeof(double) * 6, hipMemcpyDeviceToHost));
    if (dev && j.wide && j.m > 0) {
      // the device-driven full run: every eigenpair (as a complete Krylov
      // run reports it), the trace check from its finishing kernel
      double dg[3] = {0, 0, 0};
      HAPOD_HIP(hipMemcpy(dg, scratch + lay[i].hhdiag, sizeof(dg), hipMemcpyDeviceToHost));
      j.sweeps = (int32_t)j.m;
      j.wide_exhausted = true;
      j.wide_missing = 0.0;
      j.wide_noise_room = 0.0;
      j.wide_unresolved = std::max(0.0, dg[0] - dg[1]);
      j.wide_slack = 16.0 * ((double)j.m + std::sqrt((double)j.m)) * u_p * std::fabs(dg[0]);
    }
    j.sigma.assign((size_t)j.rank, 0.0);
    if (j.rank > 0)
      HAPOD_HIP(hipMemcpy(j.sigma.data(), scratch + lay[i].sigma, sizeof(double) * j.rank, hipMemcpyDeviceToHost));
    if (!j.wide && j.m > 0)
      HAPOD_HIP(hipMemcpy(&j.sweeps, scratch + lay[i].sweeps, sizeof(int32_t), hipMemcpyDeviceToHost));
    // a wide node's truncation is trusted only if the eigenpairs it did not
    // get cannot hold more than the budget eps^2 (Def. 2.5) allows
    if (j.wide && (!j.wide_exhausted || j.info[0] + j.wide_missing > j.eps * j.eps ||
                   j.info[0] + j.wide_unresolved > j.eps * j.eps + j.wide_slack + j.wide_noise_room)) {
      set_error("wide eigensolver: " + std::to_string(j.sweeps) + " Krylov steps on an m = " +
                std::to_string(j.m) + " Gram did not resolve every eigenvalue the truncation needs" +
                (j.wide_exhausted ? " (unconverged energy above the budget)" : " (step limit reached)"));
      return HAPOD_E_UNSUPPORTED;
    }
  }
  if (dev && overflow) {
    // a rank above its output's capacity: the lift stopped at the capacity;
    // the batch runs again with the ranks read back first
    bool over = false;
    for (int i = 0; i < nj; ++i) over = over || (capped[i] && jobs[i].rank > cap[i]);
    if (over) {
      for (int i = 0; i < nj; ++i)
        if (capped[i]) jobs[i].out = nullptr;
      if (out_block_mine) pool.free(out_block_mine);
      if (batch_block) *batch_block = nullptr;
      *overflow = true;
    }
  }
  if (times && ev.ok && gc) {
    // a graph launch: its phases are not separated
    float a = 0;
    if (hipEventElapsedTime(&a, ev.e[0], ev.e[4]) == hipSuccess) times->graph += a;
  } else if (times && ev.ok) {
    float a = 0;
    if (hipEventElapsedTime(&a, ev.e[0], ev.e[1]) == hipSuccess) times->gram += a;
    if (hipEventElapsedTime(&a, ev.e[1], ev.e[2]) == hipSuccess) times->eig += a;
    if (hipEventElapsedTime(&a, ev.e[2], ev.e[3]) == hipSuccess) times->trunc += a;
    if (hipEventElapsedTime(&a, ev.e[3], ev.e[4]) == hipSuccess) times->lift += a;
  }
  return HAPOD_OK;
}


// A device-driven batch sizes each batch-allocated output for the rank the
// node had in the plan's previous run (else for m); if a rank came out
// larger, the batch runs again with the ranks read back before the lift.
hapod_status run_pod_batch(hapod_precision prec, std::vector<PodJob>& jobs, int policy_small, int policy_wide,
                           int jacobi_max, Pool& pool, hipStream_t stream, PhaseTimes* times,
                           void** batch_block = nullptr, bool autotune = false, BatchStats* bstats = nullptr,
                           GraphCache* gcache = nullptr) {
  bool overflow = false;
  hapod_status st = run_pod_batch_impl(prec, jobs, policy_small, policy_wide, jacobi_max, pool, stream, times,
                                       batch_block, autotune, true, &overflow, bstats, gcache);
  if (st != HAPOD_OK || !overflow) return st;
  if (bstats) {
    --bstats->device;
    ++bstats->reruns;
  }
  st = run_pod_batch_impl(prec, jobs, policy_small, policy_wide, jacobi_max, pool, stream, times, batch_block, false,
                          false, &overflow, bstats, nullptr);
  if (bstats) --bstats->host;  // counted as a rerun only
  return st;
}

hapod_status check_prec(hapod_precision p) {
  if (p != HAPOD_FP64 && p != HAPOD_FP32 && p != HAPOD_BF16X3) {
    set_error("unknown precision");
    return HAPOD_E_INVALID;
  }
  return HAPOD_OK;
}

// Pool used by the step-level entry points (no plan).  Never destroyed: a
// static object's destructor would call hipFree from the process's exit
// handlers, after the HIP runtime (or a profiler attached to it) may already
// have been torn down; the device memory goes back with the process.
Pool& step_pool() {
  static Pool* p = new Pool;
  return *p;
}

}  // namespace

// pool callbacks for wide_eigh
void* pool_alloc_cb(void* pool, size_t bytes) {
  void* p = nullptr;
  if (static_cast<Pool*>(pool)->alloc(bytes, &p) != HAPOD_OK) return nullptr;
  return p;
}
void pool_free_cb(void* pool, void* p) { static_cast<Pool*>(pool)->free(p); }

}  // namespace hapod

using namespace hapod;

// Diagnostics of one sketched local POD.
struct SketchInfo {
  int64_t ell = 0;         // sketch columns
  double residual = 0.0;   // ||S - Q Q^T S||_F^2, computed from the residual itself
  int32_t passes_y = 0;    // Cholesky-QR passes on the sketch Y = S Omega
  int32_t passes_b = 0;    // and on B^T = S^T Q
  int32_t sweeps = 0;      // Jacobi sweeps on the small factor
  int32_t kind = 0;        // test matrix of the result: 0 sparse sign map, 1 Gaussian
  int64_t res_cols = 0;    // columns of the basis the residual product used (ell, or the rank)
  float ms[6] = {0, 0, 0, 0, 0, 0};  // sketch, orthonormalisation, B, residual, small SVD, lift
};

// ===========================================================================
// Plan
// ===========================================================================
struct hapod_plan_s {
  int32_t num_nodes = 0;
  std::vector<int32_t> parent;
  std::vector<int64_t> leaf_cols;
  int64_t n = 0;
  hapod_options opts{};
  std::vector<double> eps;
  std::vector<int32_t> level;
  std::vector<int64_t> acc;
  std::vector<std::vector<int32_t>> children;
  std::vector<std::vector<int32_t>> by_level;  // index 0 = level 1
  int32_t root = -1;
  // last run
  bool has_result = false;
  std::vector<int64_t> rank, m_in, n_neg;
  std::vector<int64_t> rank_hint;  // ranks of the previous run (device-driven output capacity)
  BatchStats bstats;               // batches of the last run
  GraphCache graphs;               // graph_levels: captured device-driven batches
  int64_t graph_captures = 0, graph_replays = 0;  // in the last run
  double graph_ms = 0.0;                          // device time of its graph launches
  std::vector<double> lam1, lam_min;
  std::vector<std::vector<double>> sigma;
  void* root_U = nullptr;  // owned by the pool
  bool root_passthrough = false;
  // per node the route of the last run (HAPOD_ROUTE_*) and the pool's peak
  std::vector<int32_t> route;
  size_t run_peak = 0;
  std::vector<const void*> root_cols;  // pass-through root: its input columns
  std::vector<int64_t> root_rbs, root_rows;
  std::vector<int64_t> rows;           // rows each node's vectors hold
  // right_vectors: per computed node its eigenvectors V[:, :N] (m x N, pool
  // block), and per inner node the children in the order of its input
  std::vector<double*> vkeep;
  std::vector<std::vector<int32_t>> in_order;
  double timing[6] = {0, 0, 0, 0, 0, 0};
  std::vector<std::array<double, 4>> level_ms;  // {gram, eig, trunc, lift} per level
  // nodes that took the sketched route: their diagnostics (ell = 0 otherwise)
  std::vector<SketchInfo> sketch;
  std::string tile_cache;  // autotune_cache, copied at plan time
  Pool pool;
};

// A column table: column j starts at p[j], row-block stride rbs[j], and
// holds rows[j] rows (rows past it read as zero).
struct Cols {
  std::vector<const void*> p;
  std::vector<int64_t> rbs, rows;
  int64_t size() const { return (int64_t)p.size(); }
  void append(const Cols& o) {
    p.insert(p.end(), o.p.begin(), o.p.end());
    rbs.insert(rbs.end(), o.rbs.begin(), o.rbs.end());
    rows.insert(rows.end(), o.rows.begin(), o.rows.end());
  }
  // m columns of A: plain column-major with leading dimension ld (a_rbs ==
  // 0), or row-block-tiled with row-block stride a_rbs (column j at
  // A + kRowBlock j elements)
  static Cols of(const void* A, int64_t ld, int64_t a_rbs, int64_t m, int64_t rows, int eb) {
    Cols c;
    c.p = a_rbs > 0 ? tiled_table(A, m, eb) : column_table(A, ld, m, eb);
    c.rbs.assign((size_t)m, a_rbs > 0 ? a_rbs : kRowBlock);
    c.rows.assign((size_t)m, rows);
    return c;
  }
};

// The conditions of the lift's guard-free dense mode for an n-row column
// table of m columns and N outputs (launch_lift_residual): every column holds
// all n rows and may be read to the next multiple of 128 rows (row-block-tiled
// with a stride of at least 128 rows per column, or n a multiple of 128),
// starts 16-byte aligned; m a multiple of 8, and ldb of 4 (or N of 128 and
// ldb of 2).
bool dense_ok(int64_t n, const Cols& A, int64_t N, int64_t ldb) {
  return dense_sizes(A.size(), N, ldb) && dense_cols(n, A.size(), A.p.data(), A.rbs.data(), A.rows.data());
}

// out = A B[:, :N] in FP64: A an n-row column table of m columns, B
// row-major m x N (ld ldb); out element (r, c) at out[c * ocs + blk_off(r,
// obs)].  Descriptors come from the pool and go back to it at once (see
// upload).
// Enqueue the upload of host bytes through the pool's staging ring; where no
// ring region was had, from `src` itself, and *wait is set: the caller then
// synchronises its stream before `src` goes away.  Blocks a helper takes
// from the pool go back to it without a synchronisation: every later use of
// them is queued on the same stream (the pool's own frees wait for the
// device).
bool upload(Pool& pool, void* dst, const void* src, size_t bytes, hipStream_t stream, bool* wait) {
  const void* s = pool.stage(src, bytes);
  if (!s) {
    s = src;
    *wait = true;
  }
  return hipMemcpyAsync(dst, s, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
}

hapod_status lift_cols(Pool& pool, int64_t n, const Cols& A, const double* B, int64_t ldb, int64_t N, double* out,
                       int64_t ocs, int64_t obs, hipStream_t stream) {
  const int64_t m = A.size();
  if (n <= 0 || m <= 0 || N <= 0) return HAPOD_OK;
  void *dc = nullptr, *dr = nullptr, *dw = nullptr, *dn = nullptr, *dk = nullptr;
  hapod_status st = HAPOD_OK;
  for (auto w : {std::make_pair(sizeof(void*) * m, &dc), std::make_pair(sizeof(int64_t) * m, &dr),
                 std::make_pair(sizeof(int64_t) * m, &dw), std::make_pair(sizeof(LiftNode), &dn),
                 std::make_pair(sizeof(int64_t), &dk)})
    if (st == HAPOD_OK) st = pool.alloc(w.first, w.second);
  LiftNode l{};
  if (st == HAPOD_OK) {
    const int64_t row_tiles = (n + kLiftTileM - 1) / kLiftTileM, col_tiles = (N + kLiftTileN - 1) / kLiftTileN;
    const int rt_per = (int)std::max<int64_t>(1, std::min<int64_t>(16, row_tiles * col_tiles / kLiftTargetItems));
    l.cols = (const void* const*)dc;
    l.rbs = (const int64_t*)dr;
    l.crows = (const int64_t*)dw;
    l.B = B;
    l.rank = (const int64_t*)dk;
    l.out = out;
    l.n = n;
    l.ldb = ldb;
    l.ocs = ocs;
    l.obs = obs;
    l.m = (int32_t)m;
    l.row_tiles = (int32_t)row_tiles;
    l.col_tiles = (int32_t)col_tiles;
    l.rt_per = rt_per;
    const int items = (int)(((row_tiles + rt_per - 1) / rt_per) * col_tiles);
    bool wait = false;
    if (!upload(pool, dc, A.p.data(), sizeof(void*) * m, stream, &wait) ||
        !upload(pool, dr, A.rbs.data(), sizeof(int64_t) * m, stream, &wait) ||
        !upload(pool, dw, A.rows.data(), sizeof(int64_t) * m, stream, &wait) ||
        !upload(pool, dn, &l, sizeof(l), stream, &wait)) {
      set_error("lift: descriptor upload failed");
      st = HAPOD_E_DEVICE;
      wait = true;
    }
    if (st == HAPOD_OK) st = launch_set_scalar_i64((int64_t*)dk, N, stream);
    if (st == HAPOD_OK)
      st = dense_ok(n, A, N, ldb) && ((uintptr_t)B & 15u) == 0 ? launch_lift_dense((const LiftNode*)dn, 1, items, stream)
                                                                 : launch_lift(0, (const LiftNode*)dn, 1, items, stream);
    if ((wait || st != HAPOD_OK) && hipStreamSynchronize(stream) != hipSuccess && st == HAPOD_OK) {
      set_error("lift: stream synchronisation failed");
      st = HAPOD_E_DEVICE;
    }
  }
  for (void* q : {dc, dr, dw, dn, dk})
    if (q) pool.free(q);
  return st;
}

// The same for A plain (a_rbs == 0, ld lda) or row-block-tiled (stride a_rbs).
hapod_status lift_fp64(Pool& pool, int64_t n, int64_t m, const double* A, int64_t lda, int64_t a_rbs, const double* B,
                       int64_t ldb, int64_t N, double* out, int64_t ocs, int64_t obs, hipStream_t stream) {
  return lift_cols(pool, n, Cols::of(A, lda, a_rbs, m, n, 8), B, ldb, N, out, ocs, obs, stream);
}

// Cross product out = L^T R in FP64 on the Gram kernel's cross mode: L and R
// n-row column tables, L's width a multiple of 128; out row-major
// (width(L) x width(R), ld ldo): out[i * ldo + j] = l_i^T r_j.  Rows are
// split into chunks (partial tiles summed in a fixed order) so that the
// launch has about 8192 work items.
hapod_status cross_cols(Pool& pool, int64_t n, const Cols& L, const Cols& R, double* out, int64_t ldo,
                        hipStream_t stream) {
  const int64_t ell = L.size(), m = R.size();
  if (ell % kGramTile != 0 || ell <= 0 || m <= 0 || n <= 0) {
    set_error("cross product: left width must be a positive multiple of 128");
    return HAPOD_E_INVALID;
  }
  const int tq = (int)(ell / kGramTile);
  const int64_t mt = ell + m;
  const int ntiles = (int)((mt + kGramTile - 1) / kGramTile);
  const int nr = ntiles - tq;
  const int pairs = tq * nr;
  const int nch = pick_chunks(n, pairs, 8192, 2048);
  const int64_t cr = ((n + nch - 1) / nch + kRowBlock - 1) / kRowBlock * kRowBlock;
  const int nchunks = (int)((n + cr - 1) / cr);
  Cols X = L;
  X.append(R);
  bool vec = (cr % 16) == 0;
  for (const void* c : X.p) vec = vec && (((uintptr_t)c & 15u) == 0);
  void *dxc = nullptr, *dxr = nullptr, *dxw = nullptr, *part = nullptr, *blob = nullptr;
  std::vector<void*> held;
  bool wait = false;  // an upload read host memory of this call directly (see upload)
  auto finish = [&](hapod_status st) {
    if (wait || st != HAPOD_OK) (void)hipStreamSynchronize(stream);
    for (void* q : held) pool.free(q);
    return st;
  };
  const std::pair<size_t, void**> want[] = {
      {sizeof(void*) * mt, &dxc}, {sizeof(int64_t) * mt, &dxr}, {sizeof(int64_t) * mt, &dxw},
      {nchunks > 1 ? sizeof(double) * (size_t)pairs * nchunks * kGramTile * kGramTile : 0, &part}};
  for (const auto& w : want) {
    if (w.first == 0) continue;
    hapod_status st = pool.alloc(w.first, w.second);
    if (st != HAPOD_OK) return finish(st);
    held.push_back(*w.second);
  }
  GramNode g{};
  g.cols = (const void* const*)dxc;
  g.rbs = (const int64_t*)dxr;
  g.crows = (const int64_t*)dxw;
  g.n = n;
  g.chunk_rows = cr;
  g.G = out;
  g.partial = (double*)part;
  g.ldg = ldo;
  g.m = (int32_t)mt;
  g.nchunks = nchunks;
  g.ntiles = ntiles;
  g.tile = kGramTile;
  g.cross = (int32_t)ell;
  // rows each tile holds (inputs of uneven height end early)
  std::vector<int64_t> tile_rows((size_t)ntiles, 0);
  for (int64_t c = 0; c < mt; ++c)
    tile_rows[(size_t)(c / kGramTile)] = std::max(tile_rows[(size_t)(c / kGramTile)], X.rows[(size_t)c]);
  // consecutive items (one XCD's concurrent workgroups) share the left tiles
  // and a run of 8 right tiles of one row chunk
  std::vector<GramItem> items;
  std::vector<int32_t> rp, rn;
  for (int c = 0; c < nchunks; ++c)
    for (int J = tq; J < ntiles; J += 8)
      for (int ti = 0; ti < tq; ++ti)
        for (int tj = J; tj < std::min(J + 8, ntiles); ++tj)
          items.push_back(GramItem{0, (int16_t)ti, (int16_t)tj, c, ti * nr + (tj - tq),
                                   std::min(tile_rows[(size_t)ti], tile_rows[(size_t)tj])});
  if (nchunks > 1)
    for (int p = 0; p < pairs; ++p) {
      rp.push_back(p);
      rn.push_back(0);
    }
  Blob bl;
  const size_t o_g = bl.add(&g, sizeof(g)), o_i = bl.add_vec(items), o_rp = bl.add_vec(rp), o_rn = bl.add_vec(rn);
  hapod_status st = pool.alloc(bl.host.size(), &blob);
  if (st != HAPOD_OK) return finish(st);
  held.push_back(blob);
  char* db = (char*)blob;
  if (!upload(pool, db, bl.host.data(), bl.host.size(), stream, &wait) ||
      !upload(pool, dxc, X.p.data(), sizeof(void*) * mt, stream, &wait) ||
      !upload(pool, dxr, X.rbs.data(), sizeof(int64_t) * mt, stream, &wait) ||
      !upload(pool, dxw, X.rows.data(), sizeof(int64_t) * mt, stream, &wait)) {
    set_error("cross product: upload failed");
    return finish(HAPOD_E_DEVICE);
  }
  const GramLaunch gl{kGramTile, vec ? 1 : 0, 0, (int32_t)items.size(), 0};
  st = launch_gram(0, (const GramNode*)(db + o_g), (const GramItem*)(db + o_i), &gl, 1, (const int32_t*)(db + o_rp),
                   (const int32_t*)(db + o_rn), (int)rp.size(), kGramTile, stream);
  return finish(st);
}

// Cholesky-QR passes Q <- Q R_p^-1 on an n x m FP64 matrix A (plain, ld lda,
// for a_rbs == 0, else row-block-tiled with row-block stride a_rbs), until
// Q^T Q is the identity to rounding.  A pass whose
// Q^T Q is not within 1/2 of the identity by Gershgorin (m max |Q^T Q - I| >
// 1/2) is shifted: Q^T Q + s I = R_p^T R_p, s = 11 (n m + m (m + 1)) u
// tr(Q^T Q), the shift of shifted Cholesky-QR (tr >= ||Q||_2^2), which lifts
// the directions A nearly lacks by about s^-1/2 per pass; the others are
// plain.  Two plain passes in a row leave Q orthonormal to rounding; after
// one plain pass the next pass's Gram already shows whether Q is (every entry
// of Q^T Q - I within 8 (sqrt(n) + m) u), and then the passes stop.  The
// first pass factors the equilibrated Gram D^-1 A^T A D^-1 (D the column
// norms), so columns of very different size (a bump far from a short leaf's
// rows is 1e-100 of its neighbours) start on equal terms: R_1 = R_1' D,
// R_1^-1 = D^-1 R_1'^-1.  A column with a zero Gram diagonal factors as a
// unit column, stays zero in every Q, and is flagged in zero[] (device, m).
// QA, QB: two row-block-tiled n x m buffers the passes alternate between (QA
// may be A itself, then overwritten).  *Q: the buffer holding the final Q.
// R (device, m x m column-major, may be null): A = Q R with R = R_p ... R_1.
hapod_status cholqr_core(Pool& pool, int64_t n, int64_t m, const double* A, int64_t lda, int64_t a_rbs, double* QA,
                         double* QB, double* R, int32_t* zero, const double** Q, int32_t* passes,
                         hipStream_t stream) {
  const size_t mm = sizeof(double) * (size_t)m * m;
  void *G = nullptr, *Rinv = nullptr, *Rk = nullptr, *Racc = nullptr, *Rtmp = nullptr, *ddev = nullptr,
       *dbad = nullptr, *dD = nullptr;
  std::vector<void*> held;
  auto finish = [&](hapod_status st) {
    (void)hipStreamSynchronize(stream);
    for (void* q : held) pool.free(q);
    return st;
  };
  const bool acc = R != nullptr;
  const std::pair<size_t, void**> want[] = {
      {mm, &G}, {mm, &Rinv}, {acc ? mm : 0, &Rk}, {acc ? mm : 0, &Racc}, {acc ? mm : 0, &Rtmp},
      {sizeof(double), &ddev}, {sizeof(int32_t) * kQrMaxPasses, &dbad}, {sizeof(double) * m, &dD}};
  for (const auto& w : want) {
    if (w.first == 0) continue;
    hapod_status st = pool.alloc(w.first, w.second);
    if (st != HAPOD_OK) return finish(st);
    held.push_back(*w.second);
  }
  hapod_status st = launch_zero_bytes(zero, sizeof(int32_t) * m, stream);
  if (st != HAPOD_OK) return finish(st);
  const double u = 1.1102230246251565e-16;
  const int64_t trbs = tiled_rbs(m);
  const double* src = A;
  int64_t src_rbs = a_rbs;
  int64_t ld = lda;
  double* dst = (QA == A) ? QB : QA;
  int plain_run = 0, pass = 0;
  // rounding of an entry of Q^T Q (n-term dot products) and of the m-term
  // triangular solve that made Q
  const double done_tol = 8.0 * (std::sqrt((double)n) + (double)m) * u;
  bool done = false;
  for (; pass < kQrMaxPasses && plain_run < 2; ++pass) {
    if ((st = gram_impl(0, 8, n, m, src, ld, (double*)G, m, stream, 0, src_rbs)) != HAPOD_OK ||
        (st = launch_gram_zero_scale((double*)G, m, m, zero, pass == 0 ? (double*)dD : nullptr, stream)) !=
            HAPOD_OK ||
        (st = launch_identity_dev((double*)G, m, m, (double*)ddev, stream)) != HAPOD_OK)
      return finish(st);
    // one readback per pass: this Gram's deviation and the previous pass's
    // Cholesky flag (after a bad pivot this Gram is meaningless, and unused)
    double dev = 0.0;
    int32_t bad_prev = 0;
    if (hipMemcpyAsync(&dev, ddev, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (pass > 0 && hipMemcpyAsync(&bad_prev, (int32_t*)dbad + pass - 1, sizeof(bad_prev), hipMemcpyDeviceToHost,
                                    stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
      set_error("Cholesky-QR: readback failed");
      return finish(HAPOD_E_DEVICE);
    }
    if (bad_prev) {
      set_error("Cholesky-QR: a Cholesky pivot was not positive (non-finite input?)");
      return finish(HAPOD_E_NUMERIC);
    }
    // the previous pass was plain and left Q^T Q within the Gram's own
    // rounding of the identity: Q is orthonormal, no further pass
    if (plain_run >= 1 && dev <= done_tol) {
      done = true;
      break;
    }
    const bool shifted = !((double)m * dev <= 0.5);
    if (shifted &&
        (st = launch_shift_diag((double*)G, m, m, 11.0 * ((double)n * m + (double)m * (m + 1)) * u, stream)) != HAPOD_OK)
      return finish(st);
    if ((st = launch_chol_inv((double*)G, m, m, (double*)Rinv, m, (int32_t*)dbad + pass, stream, 0.0)) != HAPOD_OK)
      return finish(st);
    if (acc && (st = launch_triu((double*)G, m, m, pass == 0 ? (double*)Racc : (double*)Rk, m, stream)) != HAPOD_OK)
      return finish(st);
    if (pass == 0 && (st = launch_unscale_factors(acc ? (double*)Racc : nullptr, m, (double*)Rinv, m, m, (double*)dD,
                                                  stream)) != HAPOD_OK)
      return finish(st);
    if (acc && pass > 0) {
      if ((st = launch_dgemm_nn(m, m, m, (double*)Rk, m, (double*)Racc, m, (double*)Rtmp, m, stream)) != HAPOD_OK)
        return finish(st);
      std::swap(Racc, Rtmp);
    }
    if ((st = lift_fp64(pool, n, m, src, ld, src_rbs, (double*)Rinv, m, m, dst, kRowBlock, trbs, stream)) != HAPOD_OK)
      return finish(st);
    src = dst;
    src_rbs = trbs;
    ld = n;
    dst = (dst == QA) ? QB : QA;
    plain_run = shifted ? 0 : plain_run + 1;
  }
  if (!done && pass > 0) {
    // the last pass's Cholesky flag (checked by the next readback otherwise)
    int32_t bad = 0;
    if (hipMemcpyAsync(&bad, (int32_t*)dbad + pass - 1, sizeof(bad), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      set_error("Cholesky-QR: readback failed");
      return finish(HAPOD_E_DEVICE);
    }
    if (bad) {
      set_error("Cholesky-QR: a Cholesky pivot was not positive (non-finite input?)");
      return finish(HAPOD_E_NUMERIC);
    }
  }
  if (!done && plain_run < 2) {
    set_error("Cholesky-QR did not reach an orthonormal factor in 12 passes");
    return finish(HAPOD_E_NUMERIC);
  }
  if (passes) *passes = pass;
  *Q = src;
  if (acc && hipMemcpyAsync(R, Racc, mm, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
    set_error("Cholesky-QR: copy of R failed");
    return finish(HAPOD_E_DEVICE);
  }
  return finish(HAPOD_OK);
}

// The QR route for one node with eps > 0, 0 < m <= kQrMaxM, m <= n, S plain
// column-major (n x m, ld lds) or row-block-tiled (s_tiled, n x m): S = Q R
// by cholqr_core (Q row-block-tiled: contiguous 128-row blocks stream faster
// than columns 8 n bytes apart), R's rows of zero columns cleared (singular
// value 0), the SVD R V = U_R diag(sigma) by one-sided Jacobi, the modes
// Q U_R.  With s_scratch, S (then tiled) may be overwritten: it serves as one
// of the two Q buffers.  out_for_rank(N, &out, &ocs, &obs) names where the N
// modes go (called once N is known, N > 0).
hapod_status qr_pod_core(Pool& pool, int64_t n, int64_t m, double* S, int64_t lds, bool s_tiled, bool s_scratch, double eps,
                         bool scaled, const std::function<hapod_status(int64_t, double**, int64_t*, int64_t*)>& out_for_rank,
                         std::vector<double>& sigma, int64_t* rank, int32_t* passes, int32_t* sweeps,
                         hipStream_t stream) {
  *rank = 0;
  const size_t mm = sizeof(double) * (size_t)m * m;
  void *R = nullptr, *Bm = nullptr, *dsig = nullptr, *QA = nullptr, *QB = nullptr, *dinfo = nullptr, *dzero = nullptr;
  std::vector<void*> held;
  auto finish = [&](hapod_status st) {
    (void)hipStreamSynchronize(stream);
    for (void* q : held) pool.free(q);
    return st;
  };
  const std::pair<size_t, void**> want[] = {
      {mm, &R}, {mm, &Bm}, {sizeof(double) * m, &dsig}, {s_scratch ? 0 : tiled_bytes(n, m, 8), &QA},
      {tiled_bytes(n, m, 8), &QB}, {sizeof(int32_t) * 2, &dinfo}, {sizeof(int32_t) * m, &dzero}};
  for (const auto& w : want) {
    if (w.first == 0) continue;
    hapod_status st = pool.alloc(w.first, w.second);
    if (st != HAPOD_OK) return finish(st);
    held.push_back(*w.second);
  }
  if (s_scratch) QA = S;
  const double* Q = nullptr;
  hapod_status st = cholqr_core(pool, n, m, S, lds, s_tiled ? tiled_rbs(m) : 0, (double*)QA, (double*)QB, (double*)R, (int32_t*)dzero,
                                &Q, passes, stream);
  if (st != HAPOD_OK) return finish(st);
  if ((st = launch_zero_rows((double*)R, m, m, (int32_t*)dzero, stream)) != HAPOD_OK) return finish(st);
  // one-sided Jacobi SVD of R: R V = U_R diag(sigma); B = U_R (diag(sigma))
  if ((st = launch_osj((double*)R, m, (double*)dsig, (double*)Bm, scaled ? 1 : 0, (int32_t*)dinfo, stream)) !=
      HAPOD_OK)
    return finish(st);
  int32_t info = 0;
  std::vector<double> sg((size_t)m);
  if (hipMemcpyAsync(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(sg.data(), dsig, sizeof(double) * m, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    set_error("hapod_node_pod_qr: readback failed");
    return finish(HAPOD_E_DEVICE);
  }
  if (info < 0) {
    set_error("hapod_node_pod_qr: the Jacobi SVD did not converge");
    return finish(HAPOD_E_NUMERIC);
  }
  if (sweeps) *sweeps = info;
  // Def. 2.5: the smallest N whose discarded squared singular values sum to at most eps^2
  int64_t N = m;
  double tail = 0.0;
  const double e2 = eps * eps;
  while (N > 0 && tail + sg[(size_t)N - 1] * sg[(size_t)N - 1] <= e2) {
    tail += sg[(size_t)N - 1] * sg[(size_t)N - 1];
    --N;
  }
  if (N > 0) {
    double* out = nullptr;
    int64_t ocs = 0, obs = 0;
    if ((st = out_for_rank(N, &out, &ocs, &obs)) != HAPOD_OK) return finish(st);
    if ((st = lift_fp64(pool, n, m, Q, n, tiled_rbs(m), (const double*)Bm, m, N, out, ocs, obs, stream)) != HAPOD_OK)
      return finish(st);
  }
  *rank = N;
  sigma.assign(sg.begin(), sg.begin() + N);
  return finish(HAPOD_OK);
}


// Residual energy per column: res[j] = ||r_j - Q b_j||^2 (device, m
// doubles) for Q an n-row column table (ell columns), B row-major ell x m
// (ld ldb) and R an n-row column table of m columns, by the FP64 lift's
// residual mode (the product Q B is compared tile by tile, never stored).
hapod_status residual_cols(Pool& pool, int64_t n, const Cols& Q, const double* B, int64_t ldb, const Cols& R,
                           double* res, hipStream_t stream) {
  const int64_t ell = Q.size(), m = R.size();
  if (n <= 0 || ell <= 0 || m <= 0) return HAPOD_OK;
  const int64_t row_tiles = (n + kLiftTileM - 1) / kLiftTileM, col_tiles = (m + kLiftTileN - 1) / kLiftTileN;
  const int rt_per = (int)std::max<int64_t>(1, std::min<int64_t>(16, row_tiles * col_tiles / kLiftTargetItems));
  const int64_t rgroups = (row_tiles + rt_per - 1) / rt_per;
  void *dqc = nullptr, *dqr = nullptr, *dqw = nullptr, *drc = nullptr, *drr = nullptr, *drw = nullptr,
       *rpart = nullptr, *dn = nullptr, *dk = nullptr;
  std::vector<void*> held;
  bool wait = false;  // an upload read host memory of this call directly (see upload)
  auto finish = [&](hapod_status st) {
    if (wait || st != HAPOD_OK) (void)hipStreamSynchronize(stream);
    for (void* q : held) pool.free(q);
    return st;
  };
  const std::pair<size_t, void**> want[] = {
      {sizeof(void*) * ell, &dqc}, {sizeof(int64_t) * ell, &dqr}, {sizeof(int64_t) * ell, &dqw},
      {sizeof(void*) * m, &drc}, {sizeof(int64_t) * m, &drr}, {sizeof(int64_t) * m, &drw},
      {sizeof(double) * (size_t)rgroups * 2 * m, &rpart}, {sizeof(LiftNode), &dn}, {sizeof(int64_t), &dk}};
  for (const auto& w : want) {
    hapod_status st = pool.alloc(w.first, w.second);
    if (st != HAPOD_OK) return finish(st);
    held.push_back(*w.second);
  }
  LiftNode l{};
  l.cols = (const void* const*)dqc;
  l.rbs = (const int64_t*)dqr;
  l.crows = (const int64_t*)dqw;
  l.B = B;
  l.rank = (const int64_t*)dk;
  l.n = n;
  l.ldb = ldb;
  l.m = (int32_t)ell;
  l.row_tiles = (int32_t)row_tiles;
  l.col_tiles = (int32_t)col_tiles;
  l.rt_per = rt_per;
  l.rcols = (const void* const*)drc;
  l.rrbs = (const int64_t*)drr;
  l.rrows = (const int64_t*)drw;
  l.rpart = (double*)rpart;
  auto up = [&](void* d, const void* h, size_t bytes) { return upload(pool, d, h, bytes, stream, &wait); };
  if (!up(dqc, Q.p.data(), sizeof(void*) * ell) || !up(dqr, Q.rbs.data(), sizeof(int64_t) * ell) ||
      !up(dqw, Q.rows.data(), sizeof(int64_t) * ell) || !up(drc, R.p.data(), sizeof(void*) * m) ||
      !up(drr, R.rbs.data(), sizeof(int64_t) * m) || !up(drw, R.rows.data(), sizeof(int64_t) * m) ||
      !up(dn, &l, sizeof(l))) {
    set_error("residual: upload failed");
    return finish(HAPOD_E_DEVICE);
  }
  hapod_status st = launch_set_scalar_i64((int64_t*)dk, m, stream);
  if (st == HAPOD_OK)
    st = launch_lift_residual((const LiftNode*)dn, (int)(rgroups * col_tiles), stream,
                              dense_ok(n, Q, m, ldb) && ((uintptr_t)B & 15u) == 0);
  if (st == HAPOD_OK) st = launch_sum_partials((const double*)rpart, rgroups * 2, m, res, stream);
  return finish(st);
}

// Orthonormal basis Q of an n x ell matrix Y (ell a multiple of 128; plain
// with leading dimension ldy for y_rbs == 0, else row-block-tiled with
// row-block stride y_rbs), 128 columns at a time, by block Gram-Schmidt with
// re-orthogonalisation: block b has the earlier blocks' span projected out,
// W = Y_b - Q_<b C_1 with C_1 = Q_<b^T Y_b (product and subtraction in one
// lift, [Q_<b, Y_b] [-C_1; I]), W = Q~ R_1 by cholqr_core, then the same
// projection once more on the orthonormal Q~ (its component along Q_<b,
// which R_1^-1 amplified by up to cond(W), goes back to rounding level),
// Q~ - Q_<b C_2 = Q_b R_2 by cholqr_core (two plain passes: Q~ is nearly
// orthonormal).  A block of a sketch holds about 128 consecutive directions
// of the spectrum, so its condition number is far below the whole
// sketch's, and passes of n x 128 replace passes of n x ell.  With R
// (device, ell x ell column-major, ld ell) non-null, Y = Q R: column block b
// of R is [C_1 + C_2 R_1; R_2 R_1] (rows of columns that were exactly zero
// cleared in each factor).  Q: the blocks' buffers (pool blocks appended to
// `held`, freed by the caller) as one column table.
hapod_status orth_blocks(Pool& pool, int64_t n, int64_t ell, const double* Y, int64_t ldy, int64_t y_rbs, double* R,
                         std::vector<void*>& held, Cols& Q, int32_t* passes, hipStream_t stream) {
  const int64_t B = kGramTile;
  const int nb = (int)(ell / B);
  const size_t blk = tiled_bytes(n, B, 8), bb = sizeof(double) * B * B;
  void *C = nullptr, *dzero = nullptr, *R1 = nullptr, *R2 = nullptr, *Rt = nullptr, *Mt = nullptr;
  hapod_status st = HAPOD_OK;
  const std::pair<size_t, void**> want[] = {{sizeof(double) * (size_t)(ell + B) * B, &C}, {sizeof(int32_t) * B, &dzero},
                                            {bb, &R1}, {bb, &R2}, {bb, &Rt}, {sizeof(double) * (size_t)ell * B, &Mt}};
  for (const auto& w : want) {
    if ((st = pool.alloc(w.first, w.second)) != HAPOD_OK) return st;
    held.push_back(*w.second);
  }
  if (R) HAPOD_TRY(launch_zero_bytes(R, sizeof(double) * (size_t)ell * ell, stream));
  Q = Cols{};
  if (passes) *passes = 0;
  for (int b = 0; b < nb; ++b) {
    void* buf[3] = {nullptr, nullptr, nullptr};
    for (void*& q : buf)
      if (st == HAPOD_OK) st = pool.alloc(blk, &q);
    auto drop = [&](void* keep) {
      for (void* q : buf)
        if (q && q != keep) pool.free(q);
    };
    if (st != HAPOD_OK) {
      drop(nullptr);
      return st;
    }
    const int64_t k = Q.size();
    const double* src = y_rbs > 0 ? Y + (size_t)b * B * kRowBlock : Y + (size_t)b * B * ldy;
    int64_t src_rbs = y_rbs, src_ld = ldy;
    // W = Y_b - Q_<b C_1 (C_1 = Q_<b^T Y_b) into buf[0]
    if (b > 0) {
      const Cols cur = Cols::of(src, ldy, y_rbs, B, n, 8);
      Cols X = Q;
      X.append(cur);
      if ((st = cross_cols(pool, n, Q, cur, (double*)C, B, stream)) == HAPOD_OK && R)
        st = launch_acc_transposed(R, ell, (int64_t)b * B, (const double*)C, B, k, B, stream);
      if (st == HAPOD_OK && (st = launch_neg_ident((double*)C, k, B, B, stream)) == HAPOD_OK)
        st = lift_cols(pool, n, X, (const double*)C, B, B, (double*)buf[0], kRowBlock, tiled_rbs(B), stream);
      src = (const double*)buf[0];
      src_rbs = tiled_rbs(B);
      src_ld = n;
    }
    // W = Q~ R_1; block 0 reads Y and alternates between buf[0] and buf[1],
    // later blocks start from buf[0], which may be overwritten
    const double* Qt = nullptr;
    int32_t p1 = 0, p2 = 0;
    if (st == HAPOD_OK)
      st = cholqr_core(pool, n, B, src, src_ld, src_rbs, (double*)buf[0], (double*)buf[1], (double*)R1,
                       (int32_t*)dzero, &Qt, &p1, stream);
    if (st == HAPOD_OK) st = launch_zero_rows((double*)R1, B, B, (int32_t*)dzero, stream);
    const double* Qb = Qt;
    if (b > 0 && st == HAPOD_OK) {
      // Q~ - Q_<b C_2 (C_2 = Q_<b^T Q~) into the free buffer, then Q_b R_2
      void* freeb = (Qt == (const double*)buf[0]) ? buf[1] : buf[0];
      void* other = buf[2];
      const Cols cur = Cols::of(Qt, n, tiled_rbs(B), B, n, 8);
      Cols X = Q;
      X.append(cur);
      if ((st = cross_cols(pool, n, Q, cur, (double*)C, B, stream)) == HAPOD_OK && R) {
        // C_2 R_1: C_2 row-major k x B is C_2^T column-major (B x k); (C_2 R_1)
        // row-major = R_1^T C_2^T column-major
        if ((st = launch_transpose((const double*)R1, B, B, (double*)Rt, B, stream)) == HAPOD_OK &&
            (st = launch_dgemm_nn(B, k, B, (const double*)Rt, B, (const double*)C, B, (double*)Mt, B, stream)) ==
                HAPOD_OK)
          st = launch_acc_transposed(R, ell, (int64_t)b * B, (const double*)Mt, B, k, B, stream);
      }
      if (st == HAPOD_OK && (st = launch_neg_ident((double*)C, k, B, B, stream)) == HAPOD_OK)
        st = lift_cols(pool, n, X, (const double*)C, B, B, (double*)freeb, kRowBlock, tiled_rbs(B), stream);
      if (st == HAPOD_OK)
        st = cholqr_core(pool, n, B, (const double*)freeb, n, tiled_rbs(B), (double*)freeb, (double*)other,
                         (double*)R2, (int32_t*)dzero, &Qb, &p2, stream);
      if (st == HAPOD_OK) st = launch_zero_rows((double*)R2, B, B, (int32_t*)dzero, stream);
      // diagonal block R_2 R_1
      if (st == HAPOD_OK && R)
        st = launch_dgemm_nn(B, B, B, (const double*)R2, B, (const double*)R1, B, (double*)Rt, B, stream);
    }
    if (st == HAPOD_OK && R) {
      const void* diag = (b > 0) ? Rt : R1;
      if (hipMemcpy2DAsync(R + (size_t)b * B * ell + (size_t)b * B, sizeof(double) * ell, diag, sizeof(double) * B,
                           sizeof(double) * B, B, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
        set_error("orthonormalisation: copy of a block factor failed");
        st = HAPOD_E_DEVICE;
      }
    }
    if (st != HAPOD_OK) {
      drop(nullptr);
      return st;
    }
    if (passes) *passes += p1 + p2;
    void* keep = nullptr;
    for (void* q : buf)
      if ((const double*)q == Qb) keep = q;
    drop(keep);
    held.push_back(keep);
    Q.append(Cols::of(keep, n, tiled_rbs(B), B, n, 8));
  }
  return HAPOD_OK;
}

// Sketched local POD of a wide node (FP64), for nodes whose Gram matrix
// cannot resolve the truncation (Rem. 2.3: the method of snapshots knows
// sigma_k^2 only to about u sigma_1^2).  A randomized range finder (Halko,
// Martinsson & Tropp, SIAM Review 2011, Alg. 4.1 and Sec. 5.1):
//   Y = S Omega        Omega m x ell Gaussian (counter-based, seeded)
//   Y = Q R_Y          orth_blocks: Q orthonormal to rounding
//   B = Q^T S          ell x m (cross-product mode of the Gram kernel; stored
//                      as B^T, m x ell)
//   r = ||S - Q B||_F^2  from the residual itself (residual mode of the lift)
//   B^T = Q' R'        orth_blocks; then B = R'^T Q'^T and the left singular
//                      vectors and singular values of B are those of R'^T:
//                      one-sided Jacobi on the columns of R'^T
//   U = Q U_B          (scaled: Q U_B diag(sigma))
// Truncation (Def. 2.5 with the sketch's residual counted as discarded
// energy): N = min{N' : r + sum_{k > N'} sigma_k(B)^2 <= eps^2}.  Then
// ||S - U U^T S||_F^2 = r + sum_{k > N} sigma_k(B)^2 <= eps^2 exactly (the
// residual is orthogonal to span(Q)), the property the HAPOD bounds
// (Thm. 3.3 - 3.5) use.  Every quantity is formed from S or Q themselves,
// never from S^T S, so it carries absolute errors of about u ||s_j|| per
// column instead of u sigma_1^2 per eigenvalue.  r > eps^2 (the node's rank
// exceeds what ell columns capture) fails with HAPOD_E_UNSUPPORTED.
// cols/rbs/crows: the node's input columns (host copies of device pointers).
hapod_status sketch_pod_core(Pool& pool, int64_t n, int64_t m, const std::vector<const void*>& cols,
                             const std::vector<int64_t>& rbs, const std::vector<int64_t>& crows, int64_t ell,
                             uint64_t seed, int32_t kind, double eps, bool scaled,
                             const std::function<hapod_status(int64_t, double**, int64_t*, int64_t*)>& out_for_rank,
                             std::vector<double>& sigma, int64_t* rank, SketchInfo* info, hipStream_t stream) {
  *rank = 0;
  SketchInfo si;
  si.ell = ell;
  Cols Sc;
  Sc.p = cols;
  Sc.rbs = rbs;
  Sc.rows = crows;
  const size_t ll = sizeof(double) * (size_t)ell * ell;
  void *Om = nullptr, *Y = nullptr, *Bt = nullptr, *res = nullptr, *Rb = nullptr, *M = nullptr, *UB = nullptr,
       *dsig = nullptr, *dinfo = nullptr;
  std::vector<void*> held;
  hipEvent_t ev[7] = {};
  auto finish = [&](hapod_status st) {
    (void)hipStreamSynchronize(stream);
    for (void* q : held) pool.free(q);
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
    return st;
  };
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      set_error("sketched POD: hipEventCreate failed");
      return finish(HAPOD_E_DEVICE);
    }
  void *dcols = nullptr, *drbs = nullptr, *drows = nullptr;
  const std::pair<size_t, void**> want[] = {
      {sizeof(double) * (size_t)m * ell, &Om}, {tiled_bytes(n, ell, 8), &Y}, {sizeof(double) * (size_t)m * ell, &Bt},
      {sizeof(double) * m, &res}, {ll, &Rb}, {ll, &M}, {ll, &UB}, {sizeof(double) * ell, &dsig},
      {sizeof(int32_t) * 2, &dinfo}, {sizeof(void*) * (size_t)m, &dcols}, {sizeof(int64_t) * (size_t)m, &drbs},
      {sizeof(int64_t) * (size_t)m, &drows}};
  for (const auto& w : want) {
    hapod_status st = pool.alloc(w.first, w.second);
    if (st != HAPOD_OK) return finish(st);
    held.push_back(*w.second);
  }
  const size_t held_base = held.size();
  int64_t full_rows = n;
  for (int64_t r : crows) full_rows = std::min(full_rows, r);
  if (hipMemcpyAsync(dcols, cols.data(), sizeof(void*) * m, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(drbs, rbs.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(drows, crows.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, stream) != hipSuccess) {
    set_error("sketched POD: column table upload failed");
    return finish(HAPOD_E_DEVICE);
  }
  hapod_status st = HAPOD_OK;
  // The sparse sign map first (one pass over S at memory speed instead of an
  // n x m x ell product); should its residual exceed eps^2, the Gaussian
  // test matrix (whose range captures the leading subspace with the least
  // oversampling) from the start.  Either way the residual decides, exactly.
  Cols Q;
  si.kind = (kind == 1) ? 1 : 0;
  const bool post = !scaled;
  for (;;) {
    (void)hipEventRecord(ev[0], stream);
    // ---- Y = S Omega ----------------------------------------------------------
    if (si.kind == 0) {
      if ((st = launch_sign_sketch((const void* const*)dcols, (const int64_t*)drbs, (const int64_t*)drows, n, m,
                                   full_rows, seed, ell, (double*)Y, kRowBlock, tiled_rbs(ell), stream)) != HAPOD_OK)
        return finish(st);
    } else if ((st = launch_normal_fill((double*)Om, m * ell, seed, stream)) != HAPOD_OK ||
               (st = lift_cols(pool, n, Sc, (const double*)Om, ell, ell, (double*)Y, kRowBlock, tiled_rbs(ell),
                               stream)) != HAPOD_OK) {
      return finish(st);
    }
    (void)hipEventRecord(ev[1], stream);
    // ---- Q = orth(Y) -------------------------------------------------------------
    if ((st = orth_blocks(pool, n, ell, (const double*)Y, n, tiled_rbs(ell), nullptr, held, Q, &si.passes_y,
                          stream)) != HAPOD_OK)
      return finish(st);
    (void)hipEventRecord(ev[2], stream);
    // ---- B^T = S^T Q (row-major B, ell x m) ---------------------------------------
    if ((st = cross_cols(pool, n, Q, Sc, (double*)Bt, m, stream)) != HAPOD_OK) return finish(st);
    (void)hipEventRecord(ev[3], stream);
    // unscaled modes are Q U_B[:, :N] themselves: their residual is taken
    // after the SVD, against the N kept columns (below)
    if (post) break;
    // ---- residual energy per column: ||s_j - Q b_j||^2 ------------------------------
    if ((st = residual_cols(pool, n, Q, (const double*)Bt, m, Sc, (double*)res, stream)) != HAPOD_OK)
      return finish(st);
    (void)hipEventRecord(ev[4], stream);
    if (si.kind == 1) break;
    std::vector<double> r0((size_t)m);
    if (hipMemcpyAsync(r0.data(), res, sizeof(double) * m, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      set_error("sketched POD: readback failed");
      return finish(HAPOD_E_DEVICE);
    }
    double rs0 = 0.0;
    for (double v : r0) rs0 += v;
    if (rs0 <= eps * eps) break;
    // the sparse map missed part of the range: its Q blocks go back, the
    // Gaussian takes over
    for (size_t q = held_base; q < held.size(); ++q) pool.free(held[q]);
    held.resize(held_base);
    Q = Cols{};
    si.kind = 1;
  }
  // ---- SVD of B through B^T = Q' R' -----------------------------------------------------
  Cols Qt;
  if ((st = orth_blocks(pool, m, ell, (const double*)Bt, m, 0, (double*)Rb, held, Qt, &si.passes_b, stream)) !=
      HAPOD_OK)
    return finish(st);
  if ((st = launch_transpose((const double*)Rb, ell, ell, (double*)M, ell, stream)) != HAPOD_OK ||
      (st = launch_osj((double*)M, ell, (double*)dsig, (double*)UB, scaled ? 1 : 0, (int32_t*)dinfo, stream)) !=
          HAPOD_OK)
    return finish(st);
  (void)hipEventRecord(ev[5], stream);
  std::vector<double> sg((size_t)ell), rs((size_t)m);
  int32_t jinfo = 0;
  if (hipMemcpyAsync(sg.data(), dsig, sizeof(double) * ell, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      (!post && hipMemcpyAsync(rs.data(), res, sizeof(double) * m, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
      hipMemcpyAsync(&jinfo, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    set_error("sketched POD: readback failed");
    return finish(HAPOD_E_DEVICE);
  }
  if (jinfo < 0) {
    set_error("sketched POD: the Jacobi SVD of the small factor did not converge");
    return finish(HAPOD_E_NUMERIC);
  }
  si.sweeps = jinfo;
  const double e2 = eps * eps;
  if (post) {
    // The residual of the modes U = Q U_B[:, :N] themselves: ||S - U U^T S||^2
    // = ||S - U C||^2 with C = U_B[:, :N]^T B (the coefficients, from B on
    // the small side), an n x m x N product instead of n x m x ell.  N is
    // chosen first with e2 / 64 of the budget left for the residual r of the
    // whole sketch basis (the discarded energy is r + sum_{k>N} sigma_k^2 by
    // orthogonality); the computed residual then certifies it.  Should it
    // exceed e2, r itself is taken and N set exactly (or, r above e2, the
    // route starts over with the Gaussian, or fails as the i.i.d. path does).
    auto tail_rank = [&](double r0, double budget, double* tail_out) {
      int64_t N = ell;
      double tail = r0;
      while (N > 0 && tail + sg[(size_t)N - 1] * sg[(size_t)N - 1] <= budget) {
        tail += sg[(size_t)N - 1] * sg[(size_t)N - 1];
        --N;
      }
      *tail_out = tail - r0;
      return N;
    };
    double tail = 0.0;
    int64_t N = tail_rank(0.0, e2 * (1.0 - 1.0 / 64.0), &tail);
    double* out = nullptr;
    int64_t ocs = 0, obs = 0;
    const Cols Bcols = Cols::of(Bt, m, 0, ell, m, 8);  // B^T, m x ell, column c = row c of B
    auto modes_and_residual = [&](int64_t Nk, double* rN) -> hapod_status {
      if (Nk == 0) {
        // no mode kept: the residual is all of S
        if ((st = residual_cols(pool, n, Q, (const double*)Bt, m, Sc, (double*)res, stream)) != HAPOD_OK) return st;
      } else {
        HAPOD_TRY(out_for_rank(Nk, &out, &ocs, &obs));
        HAPOD_TRY(lift_cols(pool, n, Q, (const double*)UB, ell, Nk, out, ocs, obs, stream));
        // C^T = B^T U_B[:, :N] (m x N, ld m) is C row-major: the residual's
        // operand, padded to a multiple of 8 rows (the product's guard-free
        // form) with zero rows against repeats of the first mode
        const int64_t Np = std::min<int64_t>(ell, (Nk + 7) / 8 * 8);
        HAPOD_TRY(lift_cols(pool, m, Bcols, (const double*)UB, ell, Nk, (double*)Om, m, kRowBlock, stream));
        if (Np > Nk) HAPOD_TRY(launch_zero_bytes((double*)Om + Nk * m, sizeof(double) * (size_t)(Np - Nk) * m, stream));
        (void)hipEventRecord(ev[6], stream);
        Cols U = Cols::of(out, ocs, obs == kRowBlock ? 0 : obs, Nk, n, 8);
        for (int64_t k = Nk; k < Np; ++k) {
          U.p.push_back(U.p[0]);
          U.rbs.push_back(U.rbs[0]);
          U.rows.push_back(U.rows[0]);
        }
        HAPOD_TRY(residual_cols(pool, n, U, (const double*)Om, m, Sc, (double*)res, stream));
      }
      if (hipMemcpyAsync(rs.data(), res, sizeof(double) * m, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        set_error("sketched POD: readback failed");
        return HAPOD_E_DEVICE;
      }
      double acc = 0.0;
      for (double v : rs) acc += v;
      *rN = acc;
      return HAPOD_OK;
    };
    double rN = 0.0;
    if ((st = modes_and_residual(N, &rN)) != HAPOD_OK) return finish(st);
    si.res_cols = N;
    if (!(rN <= e2)) {
      // the budget's reserve was too small: r of the whole basis decides
      if ((st = residual_cols(pool, n, Q, (const double*)Bt, m, Sc, (double*)res, stream)) != HAPOD_OK)
        return finish(st);
      if (hipMemcpyAsync(rs.data(), res, sizeof(double) * m, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        set_error("sketched POD: readback failed");
        return finish(HAPOD_E_DEVICE);
      }
      double r = 0.0;
      for (double v : rs) r += v;
      if (!(r <= e2)) {
        if (si.kind == 0) {
          // the sparse map missed part of the range: the Gaussian from the start
          if ((st = finish(HAPOD_OK)) != HAPOD_OK) return st;
          return sketch_pod_core(pool, n, m, cols, rbs, crows, ell, seed, 1, eps, scaled, out_for_rank, sigma, rank,
                                 info, stream);
        }
        si.residual = r;
        set_error("sketched POD: the residual energy " + std::to_string(r) + " of a " + std::to_string(ell) +
                  "-column sketch exceeds eps^2 = " + std::to_string(e2) +
                  " (the node's rank is beyond the sketch: use a wider sketch or the method of snapshots)");
        if (info) *info = si;
        return finish(HAPOD_E_UNSUPPORTED);
      }
      const int64_t N2 = tail_rank(r, e2, &tail);
      if (N2 != N) {
        N = N2;
        if ((st = modes_and_residual(N, &rN)) != HAPOD_OK) return finish(st);
      }
      si.res_cols = ell;
      rN = r + tail;
    }
    si.residual = std::max(0.0, rN - tail);
    (void)hipEventSynchronize(ev[6]);
    // ms: sketch, orthonormalisation, B, residual (after the modes), small SVD, modes
    float a[6] = {0, 0, 0, 0, 0, 0};
    (void)hipEventElapsedTime(&a[0], ev[0], ev[1]);
    (void)hipEventElapsedTime(&a[1], ev[1], ev[2]);
    (void)hipEventElapsedTime(&a[2], ev[2], ev[3]);
    (void)hipEventElapsedTime(&a[4], ev[3], ev[5]);
    if (N > 0) (void)hipEventElapsedTime(&a[5], ev[5], ev[6]);
    float total = 0.f;
    (void)hipEventRecord(ev[4], stream);
    (void)hipEventSynchronize(ev[4]);
    (void)hipEventElapsedTime(&total, ev[0], ev[4]);
    a[3] = std::max(0.f, total - a[0] - a[1] - a[2] - a[4] - a[5]);
    for (int k = 0; k < 6; ++k) si.ms[k] = a[k];
    *rank = N;
    sigma.assign(sg.begin(), sg.begin() + N);
    if (info) *info = si;
    return finish(HAPOD_OK);
  }
  si.res_cols = ell;
  double r2 = 0.0;
  for (double v : rs) r2 += v;
  si.residual = r2;
  if (!(r2 <= e2)) {
    set_error("sketched POD: the residual energy " + std::to_string(r2) + " of a " + std::to_string(ell) +
              "-column sketch exceeds eps^2 = " + std::to_string(e2) +
              " (the node's rank is beyond the sketch: use a wider sketch or the method of snapshots)");
    if (info) *info = si;
    return finish(HAPOD_E_UNSUPPORTED);
  }
  // Def. 2.5 with the residual as discarded energy
  int64_t N = ell;
  double tail = r2;
  while (N > 0 && tail + sg[(size_t)N - 1] * sg[(size_t)N - 1] <= e2) {
    tail += sg[(size_t)N - 1] * sg[(size_t)N - 1];
    --N;
  }
  if (N > 0) {
    double* out = nullptr;
    int64_t ocs = 0, obs = 0;
    if ((st = out_for_rank(N, &out, &ocs, &obs)) != HAPOD_OK) return finish(st);
    if ((st = lift_cols(pool, n, Q, (const double*)UB, ell, N, out, ocs, obs, stream)) != HAPOD_OK) return finish(st);
  }
  (void)hipEventRecord(ev[6], stream);
  (void)hipEventSynchronize(ev[6]);
  for (int k = 0; k < 6; ++k) (void)hipEventElapsedTime(&si.ms[k], ev[k], ev[k + 1]);
  *rank = N;
  sigma.assign(sg.begin(), sg.begin() + N);
  if (info) *info = si;
  return finish(HAPOD_OK);
}


// Device memory a run may need at most, every node keeping all its inputs
// (rank = input count, capped by its rows): per level, the outputs still
// alive (children of later levels) plus the level's own outputs and its
// batch scratch (per node Gram, eigenvectors and lift operand, m^2 doubles
// each, or the sketch's buffers on the sketched route; plus one set of
// partial tiles of the Gram work items, 8192 x 128^2 doubles).  *min_need:
// what the leaf level's scratch alone takes, which any run needs whatever
// the ranks.
size_t plan_worst_case(const hapod_plan_s& P, size_t* min_need) {
  const int eb = elem_bytes(P.opts.prec);
  const int32_t nn = P.num_nodes;
  std::vector<int64_t> width(nn, 0), in(nn, 0);
  const size_t partial = sizeof(double) * 8192 * kGramTile * kGramTile;
  auto scratch = [&](int32_t a) -> size_t {
    const size_t m = (size_t)in[a];
    const int64_t ell = P.opts.sketch_cols;
    if (ell > 0 && (int64_t)m >= 2 * ell && P.rows[a] >= ell)
      return 3 * tiled_bytes(P.rows[a], ell, 8) + 3 * sizeof(double) * m * ell;
    return 3 * sizeof(double) * m * m + (eb == 4 ? sizeof(float) * m * m : 0);
  };
  size_t worst = 0, leaf_scratch = 0;
  for (int32_t l = 0; l < (int32_t)P.by_level.size(); ++l) {
    size_t batch = 0, live = 0;
    for (int32_t a : P.by_level[l]) {
      in[a] = P.children[a].empty() ? P.leaf_cols[a] : 0;
      for (int32_t b : P.children[a]) in[a] += width[b];
      width[a] = (P.eps[a] == 0.0) ? in[a] : std::min<int64_t>(in[a], P.rows[a]);
      if (P.eps[a] == 0.0) continue;
      batch += scratch(a) + tiled_bytes(P.rows[a], width[a], eb);
      if (l == 0) leaf_scratch += scratch(a);
    }
    // outputs of computed nodes below this level whose parent is at or above it
    for (int32_t b = 0; b < nn; ++b)
      if (P.level[b] <= l && P.parent[b] >= 0 && P.level[P.parent[b]] > l && P.eps[b] > 0.0)
        live += tiled_bytes(P.rows[b], width[b], eb);
    worst = std::max(worst, live + batch + (batch ? partial : 0));
  }
  if (min_need) *min_need = leaf_scratch;
  return worst;
}

extern "C" {

const char* hapod_last_error(void) { return g_last_error.c_str(); }

hapod_status hapod_plan(const hapod_tree* tree, double eps_star, double omega, const hapod_options* opts,
                        hapod_plan_t* out) {
  if (!tree || !out || !tree->parent || !tree->leaf_cols) {
    set_error("hapod_plan: NULL argument");
    return HAPOD_E_INVALID;
  }
  if (!(eps_star >= 0.0) || !(omega >= 0.0 && omega <= 1.0) || tree->n <= 0 || tree->num_nodes <= 0) {
    set_error("hapod_plan: need eps_star >= 0, 0 <= omega <= 1, n > 0, num_nodes > 0");
    return HAPOD_E_INVALID;
  }
  if (opts) HAPOD_TRY(check_prec(opts->prec));
  if (opts && opts->block_gram && opts->prec != HAPOD_FP64) {
    // the set blocks assume children's modes orthonormal to working accuracy;
    // FP32 modes are not, and mixing exact blocks with computed FP32 ones
    // moves ranks at the noise floor far more than the rounding itself
    set_error("hapod_plan: block_gram needs the FP64 form");
    return HAPOD_E_INVALID;
  }
  if (opts && opts->qr_pod && (opts->prec != HAPOD_FP64 || opts->right_vectors)) {
    // the QR route computes in double and keeps no right singular vectors
    set_error("hapod_plan: qr_pod needs the FP64 form and excludes right_vectors");
    return HAPOD_E_INVALID;
  }
  if (opts && opts->sketch_cols != 0 &&
      (opts->prec != HAPOD_FP64 || opts->right_vectors || opts->sketch_cols < kGramTile ||
       opts->sketch_cols > kSketchMaxCols || opts->sketch_cols % kGramTile != 0)) {
    // the sketched route computes in double, keeps no right singular
    // vectors, and its sketch is whole 128-column tiles up to the Jacobi
    // SVD's 512 columns
    set_error("hapod_plan: sketch_cols needs the FP64 form, excludes right_vectors, and must be 128, 256, 384 or 512");
    return HAPOD_E_INVALID;
  }
  if (opts && opts->sketch_kind != 0 && opts->sketch_kind != 1) {
    set_error("hapod_plan: sketch_kind must be 0 (sparse sign map, Gaussian fallback) or 1 (Gaussian)");
    return HAPOD_E_INVALID;
  }
  if (opts && ((opts->leaf_layout != 0 && opts->leaf_layout != 1) ||
               (opts->leaf_passthrough != 0 && opts->leaf_passthrough != 1))) {
    set_error("hapod_plan: leaf_layout and leaf_passthrough must be 0 or 1");
    return HAPOD_E_INVALID;
  }
  auto P = std::make_unique<hapod_plan_s>();
  const int32_t nn = tree->num_nodes;
  P->num_nodes = nn;
  P->parent.assign(tree->parent, tree->parent + nn);
  P->leaf_cols.assign(tree->leaf_cols, tree->leaf_cols + nn);
  P->n = tree->n;
  if (opts) P->opts = *opts;
  else {
    P->opts.prec = HAPOD_FP64;
  }
  // ---- Def. 3.1: one root, parents in range, everything reaches the root ----
  int roots = 0;
  for (int32_t i = 0; i < nn; ++i) {
    const int32_t p = P->parent[i];
    if (p == -1) {
      ++roots;
      P->root = i;
    } else if (p < 0 || p >= nn || p == i) {
      set_error("hapod_plan: parent[" + std::to_string(i) + "] out of range");
      return HAPOD_E_TREE;
    }
  }
  if (roots != 1) {
    set_error("hapod_plan: expected exactly one root, found " + std::to_string(roots));
    return HAPOD_E_TREE;
  }
  for (int32_t i = 0; i < nn; ++i) {
    int32_t j = i, steps = 0;
    while (j != P->root) {
      j = P->parent[j];
      if (++steps > nn) {
        set_error("hapod_plan: node " + std::to_string(i) + " is on a cycle");
        return HAPOD_E_TREE;
      }
    }
  }
  P->children.assign(nn, {});
  for (int32_t i = 0; i < nn; ++i)
    if (P->parent[i] >= 0) P->children[P->parent[i]].push_back(i);
  for (int32_t i = 0; i < nn; ++i)
    if (P->children[i].empty() && P->leaf_cols[i] < 0) {
      set_error("hapod_plan: negative leaf column count");
      return HAPOD_E_INVALID;
    }
  // ---- levels (height) and |S~_alpha| by a children-first order --------------
  std::vector<int32_t> order;
  order.reserve(nn);
  {
    std::vector<std::pair<int32_t, bool>> st{{P->root, false}};
    while (!st.empty()) {
      auto [a, done] = st.back();
      st.pop_back();
      if (done) {
        order.push_back(a);
        continue;
      }
      st.push_back({a, true});
      for (auto it = P->children[a].rbegin(); it != P->children[a].rend(); ++it) st.push_back({*it, false});
    }
  }
  if (tree->leaf_rows)
    for (int32_t i = 0; i < nn; ++i)
      if (P->children[i].empty() && (tree->leaf_rows[i] < 1 || tree->leaf_rows[i] > tree->n)) {
        set_error("hapod_plan: leaf_rows outside 1..n");
        return HAPOD_E_INVALID;
      }
  P->level.assign(nn, 0);
  P->acc.assign(nn, 0);
  P->rows.assign(nn, 0);
  for (int32_t a : order) {
    int32_t lv = 0;
    int64_t cnt = 0, rw = 0;
    for (int32_t b : P->children[a]) {
      lv = std::max(lv, P->level[b]);
      cnt += P->acc[b];
      rw = std::max(rw, P->rows[b]);
    }
    P->level[a] = lv + 1;
    P->acc[a] = P->children[a].empty() ? P->leaf_cols[a] : cnt;
    P->rows[a] = P->children[a].empty() ? (tree->leaf_rows ? tree->leaf_rows[a] : tree->n) : rw;
  }
  const int32_t LT = P->level[P->root];
  P->by_level.assign(LT, {});
  for (int32_t i = 0; i < nn; ++i) P->by_level[P->level[i] - 1].push_back(i);
  // ---- Thm. 3.5 ----------------------------------------------------------------
  P->eps.assign(nn, 0.0);
  const double total = (double)P->acc[P->root];
  for (int32_t a = 0; a < nn; ++a) {
    if (a == P->root)
      P->eps[a] = std::sqrt(total) * omega * eps_star;
    else
      P->eps[a] = std::sqrt((double)P->acc[a]) / std::sqrt((double)(LT - 1)) * std::sqrt(1.0 - omega * omega) *
                  eps_star;
  }
  if (P->opts.node_eps_override)
    for (int32_t a = 0; a < nn; ++a)
      if (P->opts.node_eps_override[a] >= 0.0) P->eps[a] = P->opts.node_eps_override[a];
  P->opts.node_eps_override = nullptr;  // not kept beyond the call
  if (P->opts.autotune_cache) {
    P->tile_cache = P->opts.autotune_cache;
    load_tile_cache(P->tile_cache);
  }
  P->opts.autotune_cache = nullptr;
  if (P->opts.mem_cap_bytes > 0) {
    // the leaf level's scratch is needed whatever the ranks: a cap below it
    // can never be met
    size_t need = 0;
    (void)plan_worst_case(*P, &need);
    if (need > (size_t)P->opts.mem_cap_bytes) {
      set_error("hapod_plan: the leaf level alone needs " + std::to_string(need) + " bytes of device scratch, above " +
                "mem_cap_bytes = " + std::to_string(P->opts.mem_cap_bytes));
      return HAPOD_E_NOMEM;
    }
    P->pool.set_cap((size_t)P->opts.mem_cap_bytes);
  }
  *out = P.release();
  return HAPOD_OK;
}

hapod_status hapod_plan_workspace(hapod_plan_t P, int64_t* worst_case_bytes, int64_t* last_run_peak_bytes) {
  if (!P) {
    set_error("hapod_plan_workspace: NULL plan");
    return HAPOD_E_INVALID;
  }
  if (worst_case_bytes) *worst_case_bytes = (int64_t)plan_worst_case(*P, nullptr);
  if (last_run_peak_bytes) *last_run_peak_bytes = P->has_result ? (int64_t)P->run_peak : 0;
  return HAPOD_OK;
}

hapod_status hapod_node_route(hapod_plan_t P, int32_t node, int32_t* route) {
  if (!P || !route) {
    set_error("hapod_node_route: NULL argument");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result) {
    set_error("hapod_node_route: no completed run");
    return HAPOD_E_STATE;
  }
  const int32_t a = node < 0 ? P->root : node;
  if (a >= P->num_nodes) {
    set_error("hapod_node_route: node out of range");
    return HAPOD_E_INVALID;
  }
  *route = P->route[a];
  return HAPOD_OK;
}

hapod_status hapod_plan_query(hapod_plan_t plan, double* eps, int32_t* level, int64_t* acc) {
  if (!plan) {
    set_error("hapod_plan_query: NULL plan");
    return HAPOD_E_INVALID;
  }
  const size_t nn = plan->num_nodes;
  if (eps) std::memcpy(eps, plan->eps.data(), nn * sizeof(double));
  if (level) std::memcpy(level, plan->level.data(), nn * sizeof(int32_t));
  if (acc) std::memcpy(acc, plan->acc.data(), nn * sizeof(int64_t));
  return HAPOD_OK;
}

hapod_status hapod_right_vectors(hapod_plan_t P, double* W, int64_t ldw, void* stream_) {
  if (!P || !W) {
    set_error("hapod_right_vectors: NULL argument");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result || !P->opts.right_vectors) {
    set_error("hapod_right_vectors: no completed run of a plan made with right_vectors = 1");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  // snapshot rows: leaves in ascending node id, each leaf's columns in order
  const int32_t nn = P->num_nodes;
  std::vector<int64_t> leaf_off(nn, -1);
  int64_t total = 0;
  for (int32_t a = 0; a < nn; ++a)
    if (P->children[a].empty()) {
      leaf_off[a] = total;
      total += P->leaf_cols[a];
    }
  if (ldw < std::max<int64_t>(total, 1)) {
    set_error("hapod_right_vectors: ldw below the number of snapshots");
    return HAPOD_E_INVALID;
  }
  const int64_t Nr = P->rank[P->root];
  if (Nr <= 0) return HAPOD_OK;
  // Def. 3.9: Lambda~_rho = diag(Lambda~_beta) Lambda_rho, Lambda_alpha the
  // node's right singular vectors (its eigenvectors V[:, :N]) or the identity
  // for eps = 0.  Top-down: T_rho = I (N_rho x N_rho); a child beta whose
  // modes are input columns [c, c + N_beta) of alpha gets
  // T_beta = Lambda_alpha[c : c + N_beta, :] T_alpha; a leaf gamma's rows of
  // W are Lambda_gamma T_gamma.
  struct View {
    const double* p;
    int64_t ld;
  };
  std::vector<void*> owned;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(stream);
    for (void* q : owned) P->pool.free(q);
  };
  auto alloc_T = [&](int64_t rows, double** out) -> hapod_status {
    void* q = nullptr;
    hapod_status st = P->pool.alloc(sizeof(double) * std::max<int64_t>(rows, 1) * Nr, &q);
    if (st != HAPOD_OK) return st;
    owned.push_back(q);
    *out = (double*)q;
    return HAPOD_OK;
  };
  // rows of leaves below a child of rank 0 stay zero
  if (hipMemset2DAsync(W, sizeof(double) * ldw, 0, sizeof(double) * total, (size_t)Nr, stream) != hipSuccess) {
    set_error("hapod_right_vectors: clearing W failed");
    return HAPOD_E_DEVICE;
  }
  double* Troot = nullptr;
  hapod_status st = alloc_T(Nr, &Troot);
  if (st == HAPOD_OK) st = launch_set_identity(Troot, Nr, Nr, stream);
  std::vector<std::pair<int32_t, View>> stack{{P->root, View{Troot, Nr}}};
  while (st == HAPOD_OK && !stack.empty()) {
    const int32_t a = stack.back().first;
    const View T = stack.back().second;
    stack.pop_back();
    const bool computed = P->eps[a] > 0.0;
    const int64_t m = P->m_in[a];
    if (computed && P->rank[a] > 0 && !P->vkeep[a]) {
      set_error("hapod_right_vectors: eigenvectors of a node were not kept");
      st = HAPOD_E_INVALID;
      break;
    }
    if (P->children[a].empty()) {
      double* out = W + leaf_off[a];
      if (computed) {
        st = launch_dgemm_nn(m, Nr, P->rank[a], P->vkeep[a], m, T.p, T.ld, out, ldw, stream);
      } else {
        // Lambda = I: the rows of W are T itself
        st = (hipMemcpy2DAsync(out, sizeof(double) * ldw, T.p, sizeof(double) * T.ld, sizeof(double) * m, (size_t)Nr,
                               hipMemcpyDeviceToDevice, stream) == hipSuccess) ? HAPOD_OK : HAPOD_E_DEVICE;
      }
      continue;
    }
    const std::vector<int32_t>& order = P->in_order[a].empty() ? P->children[a] : P->in_order[a];
    int64_t c = 0;
    for (int32_t b : order) {
      const int64_t wb = P->rank[b];
      if (wb <= 0) continue;
      if (computed) {
        double* Tb = nullptr;
        st = alloc_T(wb, &Tb);
        if (st == HAPOD_OK) st = launch_dgemm_nn(wb, Nr, P->rank[a], P->vkeep[a] + c, m, T.p, T.ld, Tb, wb, stream);
        if (st != HAPOD_OK) break;
        stack.push_back({b, View{Tb, wb}});
      } else {
        stack.push_back({b, View{T.p + c, T.ld}});  // Lambda = I: a slice of T
      }
      c += wb;
    }
  }
  if (st != HAPOD_OK) {
    cleanup();
    return st;
  }
  cleanup();
  return HAPOD_OK;
}

void hapod_destroy(hapod_plan_t plan) { delete plan; }

hapod_status hapod_level_timing(hapod_plan_t P, int32_t level, double* ms4) {
  if (!P || !ms4) {
    set_error("hapod_level_timing: NULL argument");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result) {
    set_error("hapod_level_timing: no completed run");
    return HAPOD_E_STATE;
  }
  if (level < 1 || level > (int32_t)P->level_ms.size()) {
    set_error("hapod_level_timing: level out of range");
    return HAPOD_E_INVALID;
  }
  for (int i = 0; i < 4; ++i) ms4[i] = P->level_ms[level - 1][i];
  return HAPOD_OK;
}

// ===========================================================================
// Run
// ===========================================================================
hapod_status hapod_run(hapod_plan_t P, hapod_leaf_fn get_leaf, void* user, void* stream_) {
  if (!P || !get_leaf) {
    set_error("hapod_run: NULL argument");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  const hapod_precision prec = P->opts.prec;
  const int eb = elem_bytes(prec);
  const int32_t nn = P->num_nodes;
  const int jmax = P->opts.jacobi_max > 0 ? std::min<int>(P->opts.jacobi_max, kJacobiMax) : 0;
  const int wave = P->opts.leaf_wave > 0 ? P->opts.leaf_wave : INT32_MAX;
  P->has_result = false;
  for (double*& v : P->vkeep)
    if (v) {
      P->pool.free(v);
      v = nullptr;
    }
  P->vkeep.assign(P->num_nodes, nullptr);
  P->in_order.assign(P->num_nodes, {});
  if (P->root_U) {
    P->pool.free(P->root_U);
    P->root_U = nullptr;
  }
  P->root_passthrough = false;
  // the previous run's ranks size the next run's device-driven outputs
  if (P->rank.size() == (size_t)nn) P->rank_hint = P->rank;
  P->bstats = BatchStats{};
  P->graphs.on = P->opts.graph_levels != 0;
  P->graphs.next = 0;
  const int64_t cap0 = P->graphs.captures, rep0 = P->graphs.replays;
  P->graph_ms = 0.0;
  P->rank.assign(nn, 0);
  P->m_in.assign(nn, 0);
  P->n_neg.assign(nn, 0);
  P->lam1.assign(nn, 0.0);
  P->lam_min.assign(nn, 0.0);
  P->sigma.assign(nn, {});
  P->sketch.assign(nn, SketchInfo{});
  P->route.assign(nn, HAPOD_ROUTE_PASSTHROUGH);
  P->pool.reset_peak();
  for (double& t : P->timing) t = 0.0;

  // Per node: the columns it hands to its parent (pointer, row-block stride,
  // rows held) and its own buffer.  A pass-through leaf's columns are fetched
  // from the provider only when its parent's group is built.
  std::vector<std::vector<const void*>> out_cols(nn);
  std::vector<std::vector<int64_t>> out_rbs(nn), out_rows(nn);
  std::vector<void*> out_buf(nn, nullptr);
  // node outputs live in per-batch blocks: a block is freed when the last
  // node whose output it holds has been consumed
  std::vector<int> out_blk(nn, -1);
  std::vector<std::pair<void*, int>> blocks;
  auto release = [&](int32_t a) {
    const int b = out_blk[a];
    out_buf[a] = nullptr;
    out_blk[a] = -1;
    if (b >= 0 && --blocks[b].second == 0) {
      P->pool.free(blocks[b].first);
      blocks[b].first = nullptr;
    }
  };
  std::vector<char> deferred(nn, 0);
  std::vector<char> holds_leaf(nn, 0);  // output columns point into leaf data
  bool release_pending = false;          // leaves handed over since the last release call
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HAPOD_HIP(hipEventCreate(&t0));
  HAPOD_HIP(hipEventCreate(&t1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{t0, t1};
  auto release_all = [&]() {
    for (int32_t i = 0; i < nn; ++i)
      if (out_buf[i] && i != P->root) release(i);
  };
  auto fetch_leaf = [&](int32_t a, std::vector<const void*>& cols, std::vector<int64_t>& rbs,
                        std::vector<int64_t>& rows) -> hapod_status {
    const void* ptr = nullptr;
    int64_t ld = 0;
    const int32_t rc = get_leaf(user, a, &ptr, &ld, stream_);
    if (rc != 0) {
      set_error("leaf provider returned " + std::to_string(rc) + " for leaf " + std::to_string(a));
      return HAPOD_E_CALLBACK;
    }
    const bool tiled = P->opts.leaf_layout == 1;
    if (P->leaf_cols[a] > 0 && (!ptr || (!tiled && ld < P->rows[a]))) {
      set_error("leaf provider gave a NULL pointer or ld < rows for leaf " + std::to_string(a));
      return HAPOD_E_CALLBACK;
    }
    if (tiled) {
      cols = tiled_table(ptr, P->leaf_cols[a], eb);
      rbs.assign(cols.size(), tiled_rbs(P->leaf_cols[a]));
    } else {
      cols = column_table(ptr, ld, P->leaf_cols[a], eb);
      rbs.assign(cols.size(), kRowBlock);
    }
    rows.assign(cols.size(), P->rows[a]);
    return HAPOD_OK;
  };
  // one node through the QR route: its input columns gathered into a
  // row-block-tiled buffer, the modes written where the batched path would put them (plain
  // n-row columns at the root, row-block-tiled elsewhere) in a pool block of
  // their own; its time counts as Gram time
  auto qr_node = [&](int32_t a, PodJob& j, PhaseTimes& ph) -> hapod_status {
    hipEvent_t q0 = nullptr, q1 = nullptr;
    HAPOD_HIP(hipEventCreate(&q0));
    HAPOD_HIP(hipEventCreate(&q1));
    EvGuard qg{q0, q1};
    HAPOD_HIP(hipEventRecord(q0, stream));
    void *Sg = nullptr, *dc = nullptr, *dr = nullptr, *dw = nullptr;
    auto drop = [&]() {
      (void)hipStreamSynchronize(stream);
      for (void* q : {Sg, dc, dr, dw})
        if (q) P->pool.free(q);
    };
    hapod_status st = P->pool.alloc(tiled_bytes(j.n, j.m, 8), &Sg);
    if (st == HAPOD_OK) st = P->pool.alloc(sizeof(void*) * j.m, &dc);
    if (st == HAPOD_OK) st = P->pool.alloc(sizeof(int64_t) * j.m, &dr);
    if (st == HAPOD_OK) st = P->pool.alloc(sizeof(int64_t) * j.m, &dw);
    if (st == HAPOD_OK &&
        (hipMemcpyAsync(dc, j.cols.data(), sizeof(void*) * j.m, hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipMemcpyAsync(dr, j.rbs.data(), sizeof(int64_t) * j.m, hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipMemcpyAsync(dw, j.crows.data(), sizeof(int64_t) * j.m, hipMemcpyHostToDevice, stream) != hipSuccess)) {
      set_error("hapod_run: upload failed");
      st = HAPOD_E_DEVICE;
    }
    if (st == HAPOD_OK)
      st = launch_gather_cols((const void* const*)dc, (const int64_t*)dr, (const int64_t*)dw, j.n, j.m, (double*)Sg,
                              tiled_rbs(j.m), stream);
    void* outp = nullptr;
    auto out_for = [&](int64_t N, double** o, int64_t* ocs, int64_t* obs) -> hapod_status {
      const size_t bytes = j.root ? sizeof(double) * (size_t)P->n * N : tiled_bytes(j.n, N, 8);
      HAPOD_TRY(P->pool.alloc(bytes, &outp));
      if (j.root) {
        *ocs = P->n;
        *obs = kRowBlock;
        if (j.n < P->n) HAPOD_TRY(launch_zero_bytes(outp, bytes, stream));
      } else {
        *ocs = kRowBlock;
        *obs = tiled_rbs(N);
      }
      *o = (double*)outp;
      return HAPOD_OK;
    };
    std::vector<double> sg;
    int64_t N = 0;
    if (st == HAPOD_OK)
      st = qr_pod_core(P->pool, j.n, j.m, (double*)Sg, j.n, true, true, j.eps, !j.root, out_for, sg, &N, nullptr, nullptr,
                       stream);
    drop();
    if (st != HAPOD_OK) {
      if (outp) P->pool.free(outp);
      return st;
    }
    float ms = 0.f;
    (void)hipEventRecord(q1, stream);
    (void)hipEventSynchronize(q1);
    (void)hipEventElapsedTime(&ms, q0, q1);
    ph.gram += ms;
    P->rank[a] = N;
    P->sigma[a] = sg;
    P->lam1[a] = sg.empty() ? 0.0 : sg.front() * sg.front();
    P->lam_min[a] = sg.empty() ? 0.0 : sg.back() * sg.back();
    P->n_neg[a] = 0;
    out_buf[a] = outp;
    if (outp) {
      blocks.push_back({outp, 1});
      out_blk[a] = (int)blocks.size() - 1;
    }
    if (a == P->root) {
      out_cols[a] = column_table(outp, P->n, N, eb);
      out_rbs[a].assign((size_t)N, kRowBlock);
      out_rows[a].assign((size_t)N, P->n);
    } else {
      out_cols[a] = tiled_table(outp, N, eb);
      out_rbs[a].assign((size_t)N, tiled_rbs(N));
      out_rows[a].assign((size_t)N, j.n);
    }
    return HAPOD_OK;
  };
  // one wide node through the sketched route: its input columns read where
  // they are (no gather), the modes written as the batched path would put
  // them; sketch, orthonormalisation, cross product and residual count as
  // Gram time, the small SVD as eigensolve time, the final product as lift
  auto sketch_node = [&](int32_t a, PodJob& j, PhaseTimes& ph) -> hapod_status {
    void* outp = nullptr;
    auto out_for = [&](int64_t N, double** o, int64_t* ocs, int64_t* obs) -> hapod_status {
      const size_t bytes = j.root ? sizeof(double) * (size_t)P->n * N : tiled_bytes(j.n, N, 8);
      if (outp) {
        // asked again (a rank set anew after a residual check): the earlier
        // output goes back once the stream is done with it
        (void)hipStreamSynchronize(stream);
        P->pool.free(outp);
        outp = nullptr;
      }
      HAPOD_TRY(P->pool.alloc(bytes, &outp));
      if (j.root) {
        *ocs = P->n;
        *obs = kRowBlock;
        if (j.n < P->n) HAPOD_TRY(launch_zero_bytes(outp, bytes, stream));
      } else {
        *ocs = kRowBlock;
        *obs = tiled_rbs(N);
      }
      *o = (double*)outp;
      return HAPOD_OK;
    };
    std::vector<double> sg;
    int64_t N = 0;
    SketchInfo si;
    // one seed per node: reruns draw the same test matrix
    const uint64_t seed = 0x6a09e667f3bcc909ull ^ ((uint64_t)a * 0x9e3779b97f4a7c15ull);
    hapod_status st = sketch_pod_core(P->pool, j.n, j.m, j.cols, j.rbs, j.crows, P->opts.sketch_cols, seed,
                                      P->opts.sketch_kind, j.eps,
                                      !j.root, out_for, sg, &N, &si, stream);
    if (st != HAPOD_OK) {
      if (outp) P->pool.free(outp);
      return st;
    }
    ph.gram += si.ms[0] + si.ms[1] + si.ms[2] + si.ms[3];
    ph.eig += si.ms[4];
    ph.lift += si.ms[5];
    P->sketch[a] = si;
    P->rank[a] = N;
    P->sigma[a] = sg;
    P->lam1[a] = sg.empty() ? 0.0 : sg.front() * sg.front();
    P->lam_min[a] = sg.empty() ? 0.0 : sg.back() * sg.back();
    P->n_neg[a] = 0;
    out_buf[a] = outp;
    if (outp) {
      blocks.push_back({outp, 1});
      out_blk[a] = (int)blocks.size() - 1;
    }
    if (a == P->root) {
      out_cols[a] = column_table(outp, P->n, N, eb);
      out_rbs[a].assign((size_t)N, kRowBlock);
      out_rows[a].assign((size_t)N, P->n);
    } else {
      out_cols[a] = tiled_table(outp, N, eb);
      out_rbs[a].assign((size_t)N, tiled_rbs(N));
      out_rows[a].assign((size_t)N, j.n);
    }
    return HAPOD_OK;
  };
  HAPOD_HIP(hipEventRecord(t0, stream));
  PhaseTimes pt;
  const int32_t LT = (int32_t)P->by_level.size();
  P->level_ms.assign(LT, {0.0, 0.0, 0.0, 0.0});
  for (int32_t l = 0; l < LT; ++l) {
    // launch groups of this level: leaves in waves of at most `wave` nodes
    std::vector<std::vector<int32_t>> groups(1);
    int in_group = 0;
    for (int32_t a : P->by_level[l]) {
      const bool leaf = P->children[a].empty();
      if (leaf && P->eps[a] == 0.0) {  // pass-through leaf: read by its parent
        deferred[a] = 1;
        P->m_in[a] = P->leaf_cols[a];
        P->rank[a] = P->leaf_cols[a];
        P->sigma[a].assign((size_t)P->leaf_cols[a], 1.0);
        continue;
      }
      if (leaf && in_group == wave) {
        groups.emplace_back();
        in_group = 0;
      }
      groups.back().push_back(a);
      in_group += leaf ? 1 : 0;
    }
    PhaseTimes lt;
    for (auto& grp : groups) {
      std::vector<PodJob> jobs;
      std::vector<int32_t> job_node;
      bool group_fetched = false;
      for (int32_t a : grp) {
        std::vector<const void*> in;
        std::vector<int64_t> in_rbs, in_rows;
        std::vector<std::pair<int64_t, int32_t>> sblk;  // (first column, child)
        hapod_status s = HAPOD_OK;
        if (P->children[a].empty()) {
          s = fetch_leaf(a, in, in_rbs, in_rows);
          group_fetched = true;
        } else {
          // block-structured Gram: raw columns (pass-through children) first,
          // so that each computed child's scaled modes start on a tile edge
          std::vector<int32_t> order(P->children[a]);
          if (P->opts.block_gram)
            std::stable_partition(order.begin(), order.end(), [&](int32_t b) { return P->eps[b] == 0.0; });
          P->in_order[a] = order;
          for (int32_t b : order) {
            if (deferred[b]) {
              group_fetched = true;
              holds_leaf[b] = 1;
              s = fetch_leaf(b, out_cols[b], out_rbs[b], out_rows[b]);
              if (s != HAPOD_OK) break;
              deferred[b] = 0;
            }
            if (P->opts.block_gram && P->eps[b] > 0.0 && !out_cols[b].empty())
              sblk.push_back({(int64_t)in.size(), b});
            in.insert(in.end(), out_cols[b].begin(), out_cols[b].end());
            in_rbs.insert(in_rbs.end(), out_rbs[b].begin(), out_rbs[b].end());
            in_rows.insert(in_rows.end(), out_rows[b].begin(), out_rows[b].end());
          }
        }
        if (s != HAPOD_OK) {
          release_all();
          return s;
        }
        P->m_in[a] = (int64_t)in.size();
        if (P->eps[a] == 0.0) {
          // POD(S, 0) = {(1, s)}: no decomposition; the vectors pass through
          for (int32_t b : P->children[a]) holds_leaf[a] |= holds_leaf[b];
          P->rank[a] = (int64_t)in.size();
          P->sigma[a].assign(in.size(), 1.0);
          out_cols[a] = in;
          out_rbs[a] = in_rbs;
          out_rows[a] = in_rows;
          if (a == P->root) {
            P->root_passthrough = true;
            P->root_cols = in;
            P->root_rbs = in_rbs;
            P->root_rows = in_rows;
          }
          continue;
        }
        PodJob j;
        if (!sblk.empty()) {
          j.s2.assign(in.size(), 0.0);
          for (auto& bb : sblk) {
            const std::vector<double>& sg = P->sigma[bb.second];
            const int64_t len = (int64_t)out_cols[bb.second].size();
            for (int64_t k = 0; k < len && k < (int64_t)sg.size(); ++k) j.s2[bb.first + k] = sg[k] * sg[k];
            j.sblk.push_back({bb.first, bb.first + len});
          }
        }
        j.keep_v = P->opts.right_vectors != 0;
        j.pass_full = P->opts.leaf_passthrough != 0 && !j.keep_v && P->children[a].empty() && a != P->root;
        j.cap_hint = (size_t)a < P->rank_hint.size() ? P->rank_hint[a] : 0;
        j.cols = std::move(in);
        j.rbs = std::move(in_rbs);
        j.crows = std::move(in_rows);
        j.n = P->rows[a];
        j.m = (int64_t)j.cols.size();
        j.eps = P->eps[a];
        j.root = (a == P->root);
        // the root's modes go out plain column-major with n rows; every other
        // node's scaled modes stay in a row-block-tiled buffer of its own rows;
        // both are allocated once the rank is known
        j.alloc_rows = j.root ? P->n : j.n;
        j.plain_out = j.root;
        jobs.push_back(std::move(j));
        job_node.push_back(a);
      }
      // the sketched route (sketch_cols = ell) takes the computed nodes of at
      // least 2 ell inputs and ell rows, one by one
      if (P->opts.sketch_cols > 0) {
        const int64_t ell = P->opts.sketch_cols;
        std::vector<PodJob> rest;
        std::vector<int32_t> rest_node;
        for (size_t k = 0; k < jobs.size(); ++k) {
          PodJob& j = jobs[k];
          const int32_t a = job_node[k];
          if (j.m < 2 * ell || j.n < ell) {
            rest.push_back(std::move(j));
            rest_node.push_back(a);
            continue;
          }
          P->route[a] = HAPOD_ROUTE_SKETCH;
          hapod_status ks = sketch_node(a, j, lt);
          if (ks != HAPOD_OK) {
            (void)hipStreamSynchronize(stream);
            release_all();
            return ks;
          }
        }
        jobs.swap(rest);
        job_node.swap(rest_node);
      }
      // the QR route (qr_pod) takes the computed nodes it covers one by one;
      // the rest are batched below
      if (P->opts.qr_pod) {
        std::vector<PodJob> rest;
        std::vector<int32_t> rest_node;
        for (size_t k = 0; k < jobs.size(); ++k) {
          PodJob& j = jobs[k];
          const int32_t a = job_node[k];
          if (j.m <= 0 || j.m > kQrMaxM || j.m > j.n) {
            rest.push_back(std::move(j));
            rest_node.push_back(a);
            continue;
          }
          P->route[a] = HAPOD_ROUTE_QR;
          hapod_status qs = qr_node(a, j, lt);
          if (qs != HAPOD_OK) {
            (void)hipStreamSynchronize(stream);
            release_all();
            return qs;
          }
        }
        jobs.swap(rest);
        job_node.swap(rest_node);
      }
      void* blk = nullptr;
      hapod_status s = jobs.empty() ? HAPOD_OK
                                    : run_pod_batch(prec, jobs, 0, 1, jmax, P->pool, stream, &lt, &blk,
                                                    P->opts.autotune != 0, &P->bstats, &P->graphs);
      if (s != HAPOD_OK) {
        (void)hipStreamSynchronize(stream);
        if (blk) P->pool.free(blk);
        for (auto& jj : jobs)
          if (jj.vkeep) P->pool.free(jj.vkeep);
        release_all();
        return s;
      }
      for (size_t k = 0; k < jobs.size(); ++k) {
        const int32_t a = job_node[k];
        const PodJob& j = jobs[k];
        P->route[a] = HAPOD_ROUTE_SNAPSHOTS;
        P->rank[a] = j.rank;
        P->sigma[a] = j.sigma;
        P->vkeep[a] = j.vkeep;
        P->lam1[a] = j.info[1];
        P->lam_min[a] = j.info[2];
        P->n_neg[a] = (int64_t)j.info[3];
        out_buf[a] = j.out;
        if (j.out && blk) {
          if (blocks.empty() || blocks.back().first != blk) blocks.push_back({blk, 0});
          out_blk[a] = (int)blocks.size() - 1;
          ++blocks.back().second;
        }
        if (j.passed) {
          // a full-rank leaf: its own columns go up (read again by the parent)
          out_cols[a] = j.cols;
          out_rbs[a] = j.rbs;
          out_rows[a] = j.crows;
          holds_leaf[a] = 1;
          P->route[a] = HAPOD_ROUTE_FULL_LEAF;
        } else if (a == P->root) {
          out_cols[a] = column_table(j.out, P->n, j.rank, eb);
          out_rbs[a].assign((size_t)j.rank, kRowBlock);
          out_rows[a].assign((size_t)j.rank, P->n);
        } else {
          out_cols[a] = tiled_table(j.out, j.rank, eb);
          out_rbs[a].assign((size_t)j.rank, j.obs);
          out_rows[a].assign((size_t)j.rank, j.n);
        }
        if (j.rank == 0 && out_buf[a]) release(a);
      }
      // the leaves this group read are no longer needed, unless a
      // pass-through node still forwards some of their columns upward
      for (int32_t a : grp)
        for (int32_t b : P->children[a]) holds_leaf[b] = 0;
      bool leaf_refs_live = false;
      for (int32_t i = 0; i < nn && !leaf_refs_live; ++i) leaf_refs_live = holds_leaf[i] != 0;
      release_pending |= group_fetched;
      if (release_pending && !leaf_refs_live) {
        release_pending = false;
        const int32_t rc = get_leaf(user, -1, nullptr, nullptr, stream_);
        if (rc != 0) {
          set_error("leaf provider returned " + std::to_string(rc) + " for the release call");
          release_all();
          return HAPOD_E_CALLBACK;
        }
      }
      // the children of this group are consumed
      for (int32_t a : grp)
        for (int32_t b : P->children[a])
          if (out_buf[b]) release(b);
    }
    P->level_ms[l] = {lt.gram, lt.eig, lt.trunc, lt.lift};
    P->graph_ms += lt.graph;
    pt.gram += lt.gram;
    pt.eig += lt.eig;
    pt.trunc += lt.trunc;
    pt.lift += lt.lift;
  }
  HAPOD_HIP(hipEventRecord(t1, stream));
  // re-orthonormalise the root's modes
  float reorth_ms = 0.f;
  if (P->opts.reorth && !P->root_passthrough && out_buf[P->root] && P->rank[P->root] > 0) {
    hipEvent_t r0 = nullptr;
    HAPOD_HIP(hipEventCreate(&r0));
    HAPOD_HIP(hipEventRecord(r0, stream));
    int64_t bad = 0;
    hapod_status s = hapod_reorth(prec, P->n, P->rank[P->root], out_buf[P->root], P->n, &bad, stream_);
    float ms = 0;
    (void)hipEventRecord(t1, stream);
    (void)hipEventSynchronize(t1);
    (void)hipEventElapsedTime(&ms, r0, t1);
    reorth_ms = ms;
    (void)hipEventDestroy(r0);
    if (s != HAPOD_OK) {
      release_all();
      return s;
    }
  }
  HAPOD_HIP(hipStreamSynchronize(stream));
  float total_ms = 0.f;
  (void)hipEventElapsedTime(&total_ms, t0, t1);
  P->graph_captures = P->graphs.captures - cap0;
  P->graph_replays = P->graphs.replays - rep0;
  P->timing[0] = total_ms;
  P->timing[1] = pt.gram;
  P->timing[2] = pt.eig;
  P->timing[3] = pt.trunc;
  P->timing[4] = pt.lift;
  P->timing[5] = reorth_ms;
  P->root_U = out_buf[P->root];
  out_buf[P->root] = nullptr;
  release_all();
  P->run_peak = P->pool.peak();
  if (!P->tile_cache.empty() && P->opts.autotune) HAPOD_TRY(save_tile_cache(P->tile_cache));
  // the blocks freed by this run stay cached for the next one (mem_cap_bytes
  // bounds them; a failed device allocation returns them first)
  P->has_result = true;
  return HAPOD_OK;
}

hapod_status hapod_modes(hapod_plan_t P, int32_t node, void* U, int64_t ldu, double* sigma, int64_t* rank,
                         void* stream_) {
  if (!P) {
    set_error("hapod_modes: NULL plan");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result) {
    set_error("hapod_modes: no completed run");
    return HAPOD_E_STATE;
  }
  if (node == -1) node = P->root;
  if (node < 0 || node >= P->num_nodes) {
    set_error("hapod_modes: node out of range");
    return HAPOD_E_INVALID;
  }
  const int64_t N = P->rank[node];
  if (rank) *rank = N;
  if (sigma && N > 0) std::memcpy(sigma, P->sigma[node].data(), sizeof(double) * N);
  if (U) {
    if (node != P->root) {
      set_error("hapod_modes: only the root's modes are kept");
      return HAPOD_E_STATE;
    }
    if (ldu < P->n) {
      set_error("hapod_modes: ldu < n");
      return HAPOD_E_INVALID;
    }
    hipStream_t stream = (hipStream_t)stream_;
    const int eb = elem_bytes(P->opts.prec);
    if (N > 0) {
      if (P->root_passthrough) {
        void *dcols = nullptr, *drbs = nullptr, *drows = nullptr;
        HAPOD_TRY(P->pool.alloc(sizeof(void*) * N, &dcols));
        HAPOD_TRY(P->pool.alloc(sizeof(int64_t) * N, &drbs));
        HAPOD_TRY(P->pool.alloc(sizeof(int64_t) * N, &drows));
        HAPOD_HIP(hipMemcpyAsync(dcols, P->root_cols.data(), sizeof(void*) * N, hipMemcpyHostToDevice, stream));
        HAPOD_HIP(hipMemcpyAsync(drbs, P->root_rbs.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice, stream));
        HAPOD_HIP(hipMemcpyAsync(drows, P->root_rows.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice, stream));
        hapod_status s = launch_copy_cols(eb, P->n, N, (const void* const*)dcols, (const int64_t*)drbs,
                                          (const int64_t*)drows, U, ldu, stream);
        HAPOD_HIP(hipStreamSynchronize(stream));
        P->pool.free(dcols);
        P->pool.free(drbs);
        P->pool.free(drows);
        HAPOD_TRY(s);
      } else {
        HAPOD_HIP(hipMemcpy2DAsync(U, (size_t)ldu * eb, P->root_U, (size_t)P->n * eb, (size_t)P->n * eb, (size_t)N,
                                   hipMemcpyDeviceToDevice, stream));
      }
    }
    HAPOD_HIP(hipStreamSynchronize(stream));
  }
  return HAPOD_OK;
}

hapod_status hapod_sketch_stats(hapod_plan_t P, int32_t node, double* out13) {
  if (!P || !out13) {
    set_error("hapod_sketch_stats: NULL argument");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result) {
    set_error("hapod_sketch_stats: no completed run");
    return HAPOD_E_STATE;
  }
  const int32_t a = node < 0 ? P->root : node;
  if (a >= P->num_nodes || P->sketch[a].ell == 0) {
    set_error("hapod_sketch_stats: the node did not take the sketched route");
    return HAPOD_E_STATE;
  }
  const SketchInfo& k = P->sketch[a];
  const double v[13] = {(double)k.ell, k.residual, (double)k.passes_y, (double)k.passes_b, (double)k.sweeps,
                        k.ms[0], k.ms[1], k.ms[2], k.ms[3], k.ms[4], k.ms[5], (double)k.kind, (double)k.res_cols};
  std::memcpy(out13, v, sizeof(v));
  return HAPOD_OK;
}

hapod_status hapod_node_stats(hapod_plan_t P, int64_t* m_in, int64_t* n_negative, double* lambda1,
                              double* lambda_min) {
  if (!P) {
    set_error("hapod_node_stats: NULL plan");
    return HAPOD_E_INVALID;
  }
  if (!P->has_result) {
    set_error("hapod_node_stats: no completed run");
    return HAPOD_E_STATE;
  }
  const size_t nn = P->num_nodes;
  if (m_in) std::memcpy(m_in, P->m_in.data(), nn * sizeof(int64_t));
  if (n_negative) std::memcpy(n_negative, P->n_neg.data(), nn * sizeof(int64_t));
  if (lambda1) std::memcpy(lambda1, P->lam1.data(), nn * sizeof(double));
  if (lambda_min) std::memcpy(lambda_min, P->lam_min.data(), nn * sizeof(double));
  return HAPOD_OK;
}

hapod_status hapod_plan_batch_stats(hapod_plan_t P, int64_t* out3) {
  if (!P || !out3) {
    set_error("hapod_plan_batch_stats: NULL argument");
    return HAPOD_E_INVALID;
  }
  out3[0] = P->bstats.device;
  out3[1] = P->bstats.host;
  out3[2] = P->bstats.reruns;
  return HAPOD_OK;
}

hapod_status hapod_plan_graph_stats(hapod_plan_t P, int64_t* out2, double* graph_ms) {
  if (!P || !out2) {
    set_error("hapod_plan_graph_stats: NULL argument");
    return HAPOD_E_INVALID;
  }
  out2[0] = P->graph_captures;
  out2[1] = P->graph_replays;
  if (graph_ms) *graph_ms = P->graph_ms;
  return HAPOD_OK;
}

hapod_status hapod_run_timing(hapod_plan_t P, double* ms6) {
  if (!P || !ms6) {
    set_error("hapod_run_timing: NULL argument");
    return HAPOD_E_INVALID;
  }
  std::memcpy(ms6, P->timing, sizeof(P->timing));
  return HAPOD_OK;
}

// ===========================================================================
// Step-level entry points
// ===========================================================================
hapod_status hapod_gram(hapod_precision prec, int64_t n, int64_t m, const void* S, int64_t lds, double* G,
                        int64_t ldg, void* stream_) {
  HAPOD_TRY(check_prec(prec));
  return gram_impl(compute_mode(prec), elem_bytes(prec), n, m, S, lds, G, ldg, (hipStream_t)stream_);
}

}  // extern "C"

namespace hapod {
// in_rbs > 0: S is row-block-tiled (column j at S + kRowBlock j elements,
// row-block stride in_rbs) instead of plain with leading dimension lds
hapod_status gram_impl(int compute, int eb, int64_t n, int64_t m, const void* S, int64_t lds, double* G, int64_t ldg,
                       hipStream_t stream, int tile_override, int64_t in_rbs) {
  if (n < 0 || m < 0 || (m > 0 && (!G || (n > 0 && !S))) || lds < std::max<int64_t>(n, 1) ||
      ldg < std::max<int64_t>(m, 1)) {
    set_error("hapod_gram: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (m == 0) return HAPOD_OK;
  if (m > 65535) {
    set_error("hapod_gram: m too large");
    return HAPOD_E_UNSUPPORTED;
  }
  Pool& pool = step_pool();
  auto cols = in_rbs > 0 ? tiled_table(S, m, eb) : column_table(S, lds, m, eb);
  int tile = tile_override > 0 ? tile_override : gram_tile_for(m);
  // split-BF16 above 256 columns: pre-split twin and 256-column tiles, as in
  // the level batches
  if (tile_override <= 0 && compute == 2 && m > kStageSplitMaxCols && n > 0) tile = 256;
  // split-BF16 at 129 .. 256 columns on 128-column tiles: one 256-column tile
  // staged from the FP32 columns, as the level batches run it (so the tile
  // tuner times what the batches would run)
  const bool own256 = (compute == 2 && tile == 128 && m > 128 && m <= kStageSplitMaxCols && n > 0);
  if (own256) tile = 256;
  const int nt = (int)((m + tile - 1) / tile);
  const int pairs = nt * (nt + 1) / 2;
  const int KB = (compute == 2) ? 32 : 16;
  // the level batches' work-item goal (8192, measured there on 2^20- and
  // 2^22-row nodes); short inputs (the sketched route's B^T, 8192 rows) take
  // chunks down to 256 rows, so that a one-tile Gram is not 4 workgroups
  // each over 2048 rows (0.25 ms of latency per Cholesky-QR pass)
  int nch = (n > 0) ? pick_chunks(n, pairs, std::max(8192, pairs), std::max<int64_t>(256, std::min<int64_t>(2048, n / 64)))
                    : 1;
  int64_t cr = (n > 0) ? ((n + nch - 1) / nch + kRowBlock - 1) / kRowBlock * kRowBlock : kRowBlock;
  nch = (n > 0) ? (int)((n + cr - 1) / cr) : 1;
  bool vec_ok = (cr % KB == 0);
  for (auto c : cols)
    if ((uintptr_t)c & 15u) vec_ok = false;
  void *dcols = nullptr, *dpart = nullptr, *dblob = nullptr, *drbs = nullptr, *drows = nullptr;
  HAPOD_TRY(pool.alloc(sizeof(void*) * m, &dcols));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * m, &drbs));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * m, &drows));
  HAPOD_TRY(launch_fill_i64((int64_t*)drbs, in_rbs > 0 ? in_rbs : kRowBlock, m, stream));
  HAPOD_TRY(launch_fill_i64((int64_t*)drows, n, m, stream));
  const int slots = nch * gram_slots_per_chunk(tile);
  if (slots > 1) HAPOD_TRY(pool.alloc(sizeof(double) * pairs * slots * tile * tile, &dpart));
  // split-BF16 with several column tiles: read a split twin (as the level batch does)
  void* dsplit = nullptr;
  const int gc = (compute == 2 && m < kBf16MinCols) ? 1 : compute;
  const bool presplit = (gc == 2 && !own256 && (tile != 128 || m > kStageSplitMaxCols) && n > 0);
  std::vector<const void*> cols_g = cols;
  std::vector<int64_t> rbs_g;
  if (presplit) {
    HAPOD_TRY(pool.alloc(tiled_bytes(n, m, 4), &dsplit));
    cols_g = tiled_table(dsplit, m, 4);
    rbs_g.assign((size_t)m, tiled_rbs(m));
  }
  void *dcols_g = nullptr, *drbs_g = nullptr;
  if (presplit) {
    HAPOD_TRY(pool.alloc(sizeof(void*) * m, &dcols_g));
    HAPOD_TRY(pool.alloc(sizeof(int64_t) * m, &drbs_g));
  }
  GramNode g{};
  g.cols = (const void* const*)(presplit ? dcols_g : dcols);
  g.rbs = (const int64_t*)(presplit ? drbs_g : drbs);
  g.crows = (const int64_t*)drows;  // the split twin holds n rows as well
  g.split = presplit ? 1 : 0;
  g.n = n;
  g.chunk_rows = cr;
  g.G = G;
  g.partial = (double*)dpart;
  g.ldg = ldg;
  g.m = (int32_t)m;
  g.nchunks = nch;
  g.ntiles = nt;
  g.pair_base = 0;
  g.tile = tile;
  std::vector<GramItem> items;
  std::vector<int32_t> rp, rn;
  int p = 0;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = ti; tj < nt; ++tj, ++p) {
      for (int c = 0; c < nch; ++c) items.push_back(GramItem{0, (int16_t)ti, (int16_t)tj, c, p});
      if (slots > 1) {
        rp.push_back(p);
        rn.push_back(0);
      }
    }
  Blob blob;
  const size_t o_c = blob.add_vec(cols), o_g = blob.add(&g, sizeof(g)), o_i = blob.add_vec(items),
               o_rp = blob.add_vec(rp), o_rn = blob.add_vec(rn);
  HAPOD_TRY(pool.alloc(blob.host.size(), &dblob));
  char* db = (char*)dblob;
  hapod_status st = HAPOD_OK;
  bool wait = false;  // (the stream is synchronised below in any case)
  do {
    // queued behind the caller's earlier work rather than waiting for it
    if (!upload(pool, db, blob.host.data(), blob.host.size(), stream, &wait) ||
        hipMemcpyAsync(dcols, db + o_c, sizeof(void*) * m, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      set_error("hapod_gram: descriptor upload failed");
      st = HAPOD_E_DEVICE;
      break;
    }
    if (presplit) {
      if (hipMemcpy(dcols_g, cols_g.data(), sizeof(void*) * m, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(drbs_g, rbs_g.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hapod_gram: descriptor upload failed");
        st = HAPOD_E_DEVICE;
        break;
      }
      st = launch_split_cols(n, m, (const void* const*)dcols, (const int64_t*)drbs, (const int64_t*)drows,
                             (float*)dsplit, stream);
      if (st != HAPOD_OK) break;
    }
    if (n == 0) {
      if (hipMemset2DAsync(G, ldg * sizeof(double), 0, m * sizeof(double), m, stream) != hipSuccess) {
        set_error("hapod_gram: memset failed");
        st = HAPOD_E_DEVICE;
      }
      break;
    }
    const int vec_mode = own256 ? 3 : (gc == 2 && tile >= 128) ? 2 : (vec_ok ? 1 : 0);
    const GramLaunch gl{tile, vec_mode, 0, (int32_t)items.size(), gc != compute ? gc : -1};
    st = launch_gram(compute, (const GramNode*)(db + o_g), (const GramItem*)(db + o_i), &gl, 1,
                     (const int32_t*)(db + o_rp), (const int32_t*)(db + o_rn), (int)rp.size(), tile, stream);
  } while (0);
  (void)hipStreamSynchronize(stream);
  pool.free(dcols);
  pool.free(drbs);
  pool.free(dpart);
  pool.free(dblob);
  pool.free(dsplit);
  pool.free(dcols_g);
  pool.free(drbs_g);
  pool.free(drows);
  return st;
}
}  // namespace hapod

extern "C" {

hapod_status hapod_eigh(int64_t m, double* G, int64_t ldg, double* lambda, double* V, int64_t ldv, int32_t* sweeps,
                        void* stream_) {
  if (m < 0 || (m > 0 && (!G || !lambda || !V)) || ldg < std::max<int64_t>(m, 1) || ldv < std::max<int64_t>(m, 1)) {
    set_error("hapod_eigh: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (m == 0) return HAPOD_OK;
  if (m > HAPOD_EIG_MAX) {
    set_error("hapod_eigh: m above HAPOD_EIG_MAX");
    return HAPOD_E_UNSUPPORTED;
  }
  hipStream_t stream = (hipStream_t)stream_;
  Pool& pool = step_pool();
  if (m > kJacobiMax) {
    WideResult wr;
    HAPOD_TRY(wide_eigh(G, ldg, m, lambda, V, ldv, std::ldexp(1.0, -53), &pool_alloc_cb, &pool_free_cb,
                        &pool, stream, &wr));
    HAPOD_HIP(hipStreamSynchronize(stream));
    if (sweeps) *sweeps = wr.iterations;
    return HAPOD_OK;
  }
  void *work = nullptr, *vwork = nullptr, *dn = nullptr, *dsw = nullptr;
  if (m > kJacobiLdsMax) HAPOD_TRY(pool.alloc(sizeof(double) * jacobi_work_doubles((int)m), &work));
  HAPOD_TRY(pool.alloc(sizeof(double) * jacobi_vwork_doubles((int)m), &vwork));
  HAPOD_TRY(pool.alloc(sizeof(EigNode), &dn));
  HAPOD_TRY(pool.alloc(sizeof(int32_t), &dsw));
  EigNode e{};
  e.G = G;
  e.work = (double*)work;
  e.Vwork = (double*)vwork;
  e.lambda = lambda;
  e.V = V;
  e.ldg = ldg;
  e.ldv = ldv;
  e.m = (int32_t)m;
  e.sweeps = (int32_t*)dsw;
  hapod_status st = HAPOD_OK;
  if (hipMemcpy(dn, &e, sizeof(e), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("hapod_eigh: descriptor upload failed");
    st = HAPOD_E_DEVICE;
  } else {
    st = launch_jacobi((const EigNode*)dn, 1, (int)m, stream);
  }
  (void)hipStreamSynchronize(stream);
  if (st == HAPOD_OK && sweeps) (void)hipMemcpy(sweeps, dsw, sizeof(int32_t), hipMemcpyDeviceToHost);
  pool.free(work);
  pool.free(vwork);
  pool.free(dn);
  pool.free(dsw);
  return st;
}

hapod_status hapod_truncate(int64_t m, const double* lambda, double eps, int64_t* rank, double* info, void* stream_) {
  if (m < 0 || (m > 0 && !lambda) || !rank || !(eps >= 0.0)) {
    set_error("hapod_truncate: bad argument");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  Pool& pool = step_pool();
  void *dn = nullptr, *dsig = nullptr, *drank = nullptr, *dinfo = nullptr;
  HAPOD_TRY(pool.alloc(sizeof(TruncNode), &dn));
  HAPOD_TRY(pool.alloc(sizeof(double) * std::max<int64_t>(m, 1), &dsig));
  HAPOD_TRY(pool.alloc(sizeof(int64_t), &drank));
  HAPOD_TRY(pool.alloc(sizeof(double) * 8, &dinfo));
  TruncNode t{};
  t.lambda = lambda;
  t.V = nullptr;
  t.B = nullptr;
  t.sigma = (double*)dsig;
  t.rank = (int64_t*)drank;
  t.info = (double*)dinfo;
  t.eps2 = eps * eps;
  t.m = (int32_t)m;
  t.policy = 0;
  hapod_status st = HAPOD_OK;
  if (hipMemcpy(dn, &t, sizeof(t), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("hapod_truncate: descriptor upload failed");
    st = HAPOD_E_DEVICE;
  } else {
    st = launch_truncate((const TruncNode*)dn, 1, stream);
  }
  (void)hipStreamSynchronize(stream);
  if (st == HAPOD_OK) {
    double inf[6];
    (void)hipMemcpy(rank, drank, sizeof(int64_t), hipMemcpyDeviceToHost);
    (void)hipMemcpy(inf, dinfo, sizeof(inf), hipMemcpyDeviceToHost);
    if (info) {
      info[0] = inf[0];
      info[1] = inf[1];
      info[2] = inf[2];
      info[3] = inf[3];
    }
  }
  pool.free(dn);
  pool.free(dsig);
  pool.free(drank);
  pool.free(dinfo);
  return st;
}

hapod_status hapod_lift(hapod_precision prec, int64_t n, int64_t m, int64_t N, const void* S, int64_t lds,
                        const double* V, int64_t ldv, const double* lambda, void* out, int64_t ldo, void* stream_) {
  HAPOD_TRY(check_prec(prec));
  if (n < 0 || m < 0 || N < 0 || N > std::max<int64_t>(m, 0) || lds < std::max<int64_t>(n, 1) ||
      ldv < std::max<int64_t>(m, 1) || ldo < std::max<int64_t>(n, 1) ||
      (n > 0 && m > 0 && N > 0 && (!S || !V || !out))) {
    set_error("hapod_lift: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (n == 0 || N == 0) return HAPOD_OK;
  hipStream_t stream = (hipStream_t)stream_;
  const int eb = elem_bytes(prec);
  Pool& pool = step_pool();
  auto cols = column_table(S, lds, m, eb);
  void *dcols = nullptr, *dB = nullptr, *dB32 = nullptr, *drank = nullptr, *dn = nullptr, *drbs = nullptr,
       *drows = nullptr;
  HAPOD_TRY(pool.alloc(sizeof(void*) * std::max<int64_t>(m, 1), &dcols));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * std::max<int64_t>(m, 1), &drbs));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * std::max<int64_t>(m, 1), &drows));
  HAPOD_TRY(launch_fill_i64((int64_t*)drbs, kRowBlock, m, stream));
  HAPOD_TRY(launch_fill_i64((int64_t*)drows, n, m, stream));
  // FP64: the operand's rows padded to whole runs of 4, for the dense lift
  const int64_t ldbB = (prec == HAPOD_FP64) ? (N + 3) / 4 * 4 : N;
  HAPOD_TRY(pool.alloc(sizeof(double) * std::max<int64_t>(m * ldbB, 1), &dB));
  if (prec != HAPOD_FP64) HAPOD_TRY(pool.alloc(sizeof(float) * std::max<int64_t>(m * N, 1), &dB32));
  void* dBs = nullptr;
  if (prec == HAPOD_BF16X3) HAPOD_TRY(pool.alloc(std::max<size_t>(split_operand_bytes(m), 128), &dBs));
  HAPOD_TRY(pool.alloc(sizeof(int64_t), &drank));
  HAPOD_TRY(pool.alloc(sizeof(LiftNode), &dn));
  LiftNode l{};
  l.cols = (const void* const*)dcols;
  l.rbs = (const int64_t*)drbs;
  l.crows = (const int64_t*)drows;
  l.B = (const double*)dB;
  l.B32 = (const float*)dB32;
  l.Bs = (char*)dBs;
  l.rank = (const int64_t*)drank;
  l.out = out;
  l.n = n;
  l.ldb = ldbB;
  l.ocs = ldo;
  l.obs = kRowBlock;
  l.m = (int32_t)m;
  l.row_tiles = (int32_t)((n + kLiftTileM - 1) / kLiftTileM);
  l.col_tiles = (int32_t)((N + kLiftTileN - 1) / kLiftTileN);
  l.item_base = 0;
  hapod_status st = HAPOD_OK;
  do {
    if (m == 0) {  // S V with no columns: zero output
      if (hipMemset2DAsync(out, ldo * eb, 0, n * eb, N, stream) != hipSuccess) st = HAPOD_E_DEVICE;
      break;
    }
    if (hipMemcpy(dcols, cols.data(), sizeof(void*) * m, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dn, &l, sizeof(l), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("hapod_lift: descriptor upload failed");
      st = HAPOD_E_DEVICE;
      break;
    }
    st = launch_lift_operand(V, ldv, lambda, m, N, (double*)dB, (float*)dB32, ldbB, stream);
    if (st != HAPOD_OK) break;
    st = launch_set_scalar_i64((int64_t*)drank, N, stream);
    if (st != HAPOD_OK) break;
    if (dBs) {
      st = launch_split_operand((const LiftNode*)dn, 1, m, stream);
      if (st != HAPOD_OK) break;
    }
    const bool dense = prec == HAPOD_FP64 && dense_sizes(m, N, ldbB) &&
                       dense_cols(n, m, cols.data(), std::vector<int64_t>((size_t)m, kRowBlock).data(),
                                  std::vector<int64_t>((size_t)m, n).data());
    st = dense ? launch_lift_dense((const LiftNode*)dn, 1, l.row_tiles * l.col_tiles, stream)
               : launch_lift(prec == HAPOD_FP64 ? 0 : (dBs ? 2 : 1), (const LiftNode*)dn, 1, l.row_tiles * l.col_tiles,
                             stream);
  } while (0);
  (void)hipStreamSynchronize(stream);
  pool.free(dcols);
  pool.free(drbs);
  pool.free(drows);
  pool.free(dB);
  if (dB32) pool.free(dB32);
  if (dBs) pool.free(dBs);
  pool.free(drank);
  pool.free(dn);
  return st;
}

hapod_status hapod_reorth(hapod_precision prec, int64_t n, int64_t N, void* U, int64_t ldu, int64_t* bad,
                          void* stream_) {
  HAPOD_TRY(check_prec(prec));
  if (n < 0 || N < 0 || ldu < std::max<int64_t>(n, 1) || (n > 0 && N > 0 && !U)) {
    set_error("hapod_reorth: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (N > 1024) {
    set_error("hapod_reorth: N above 1024");
    return HAPOD_E_UNSUPPORTED;
  }
  if (bad) *bad = 0;
  if (n == 0 || N == 0) return HAPOD_OK;
  hipStream_t stream = (hipStream_t)stream_;
  const int eb = elem_bytes(prec);
  Pool& pool = step_pool();
  void *W = nullptr, *Rinv = nullptr, *Rinv32 = nullptr, *tmp = nullptr, *dcols = nullptr, *dn = nullptr,
       *drank = nullptr,
       *dbad = nullptr, *drbs = nullptr, *drows = nullptr;
  HAPOD_TRY(pool.alloc(sizeof(double) * N * N, &W));
  HAPOD_TRY(pool.alloc(sizeof(double) * N * N, &Rinv));
  HAPOD_TRY(pool.alloc(sizeof(float) * N * N, &Rinv32));
  HAPOD_TRY(pool.alloc((size_t)n * N * eb, &tmp));
  HAPOD_TRY(pool.alloc(sizeof(void*) * N, &dcols));
  HAPOD_TRY(pool.alloc(sizeof(LiftNode), &dn));
  HAPOD_TRY(pool.alloc(sizeof(int64_t), &drank));
  HAPOD_TRY(pool.alloc(sizeof(int32_t), &dbad));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * N, &drbs));
  HAPOD_TRY(pool.alloc(sizeof(int64_t) * N, &drows));
  HAPOD_TRY(launch_fill_i64((int64_t*)drbs, kRowBlock, N, stream));
  HAPOD_TRY(launch_fill_i64((int64_t*)drows, n, N, stream));
  hapod_status st = HAPOD_OK;
  int64_t total_bad = 0;
  auto cols = column_table(U, ldu, N, eb);
  for (int pass = 0; pass < 2 && st == HAPOD_OK; ++pass) {
    // W = U^T U accumulated in FP64
    st = gram_impl(prec == HAPOD_FP64 ? 0 : 3, eb, n, N, U, ldu, (double*)W, N, stream);
    if (st != HAPOD_OK) break;
    st = launch_chol_inv((double*)W, N, N, (double*)Rinv, N, (int32_t*)dbad, stream);
    if (st != HAPOD_OK) break;
    LiftNode l{};
    l.cols = (const void* const*)dcols;
    l.rbs = (const int64_t*)drbs;
    l.crows = (const int64_t*)drows;
    l.B = (const double*)Rinv;
    l.B32 = (const float*)Rinv32;
    if (prec != HAPOD_FP64) {
      st = launch_to_f32((const double*)Rinv, (float*)Rinv32, N * N, stream);
      if (st != HAPOD_OK) break;
    }
    l.rank = (const int64_t*)drank;
    l.out = tmp;
    l.n = n;
    l.ldb = N;
    l.ocs = n;
    l.obs = kRowBlock;
    l.m = (int32_t)N;
    l.row_tiles = (int32_t)((n + kLiftTileM - 1) / kLiftTileM);
    l.col_tiles = (int32_t)((N + kLiftTileN - 1) / kLiftTileN);
    if (hipMemcpyAsync(dcols, cols.data(), sizeof(void*) * N, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(dn, &l, sizeof(l), hipMemcpyHostToDevice, stream) != hipSuccess) {
      set_error("hapod_reorth: upload failed");
      st = HAPOD_E_DEVICE;
      break;
    }
    st = launch_set_scalar_i64((int64_t*)drank, N, stream);
    if (st != HAPOD_OK) break;
    st = launch_lift(prec == HAPOD_FP64 ? 0 : 1, (const LiftNode*)dn, 1, l.row_tiles * l.col_tiles, stream);
    if (st != HAPOD_OK) break;
    if (hipMemcpy2DAsync(U, ldu * eb, tmp, n * eb, n * eb, N, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      set_error("hapod_reorth: copy back failed");
      st = HAPOD_E_DEVICE;
      break;
    }
    int32_t nb = 0;
    (void)hipStreamSynchronize(stream);
    (void)hipMemcpy(&nb, dbad, sizeof(int32_t), hipMemcpyDeviceToHost);
    total_bad = std::max<int64_t>(total_bad, nb);
  }
  (void)hipStreamSynchronize(stream);
  if (bad) *bad = total_bad;
  for (void* p : {W, Rinv, Rinv32, tmp, dcols, dn, drank, dbad, drbs, drows}) pool.free(p);
  return st;
}

hapod_status hapod_node_pod(hapod_precision prec, int64_t n, int64_t m, const void* S, int64_t lds, double eps,
                            int32_t scaled, void* out, int64_t ldo, double* sigma, int64_t* rank, void* stream_) {
  HAPOD_TRY(check_prec(prec));
  if (n < 0 || m < 0 || !(eps >= 0.0) || !rank || lds < std::max<int64_t>(n, 1) || ldo < std::max<int64_t>(n, 1) ||
      (n > 0 && m > 0 && (!S || !out))) {
    set_error("hapod_node_pod: bad argument");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  const int eb = elem_bytes(prec);
  if (eps == 0.0) {  // POD(S, 0) = {(1, s)}
    if (n > 0 && m > 0)
      HAPOD_HIP(hipMemcpy2DAsync(out, ldo * eb, S, lds * eb, n * eb, m, hipMemcpyDeviceToDevice, stream));
    HAPOD_HIP(hipStreamSynchronize(stream));
    *rank = m;
    if (sigma)
      for (int64_t i = 0; i < m; ++i) sigma[i] = 1.0;
    return HAPOD_OK;
  }
  if (m == 0 || n == 0) {
    *rank = 0;
    return HAPOD_OK;
  }
  std::vector<PodJob> jobs(1);
  jobs[0].cols = column_table(S, lds, m, eb);
  jobs[0].rbs.assign((size_t)m, kRowBlock);
  jobs[0].crows.assign((size_t)m, n);
  jobs[0].n = n;
  jobs[0].m = m;
  jobs[0].eps = eps;
  jobs[0].root = (scaled == 0);
  jobs[0].out = out;
  jobs[0].ocs = ldo;
  jobs[0].obs = kRowBlock;
  HAPOD_TRY(run_pod_batch(prec, jobs, 0, 1, 0, step_pool(), stream, nullptr));
  *rank = jobs[0].rank;
  if (sigma && jobs[0].rank > 0) std::memcpy(sigma, jobs[0].sigma.data(), sizeof(double) * jobs[0].rank);
  return HAPOD_OK;
}

hapod_status hapod_plan_node_pod(hapod_plan_t P, int32_t node, const void* S, int64_t lds, int64_t m, void* out,
                                 int64_t ldo, double* sigma, int64_t* rank, void* stream_) {
  if (!P || !rank) {
    set_error("hapod_plan_node_pod: NULL argument");
    return HAPOD_E_INVALID;
  }
  const int32_t a = node < 0 ? P->root : node;
  if (a >= P->num_nodes) {
    set_error("hapod_plan_node_pod: node out of range");
    return HAPOD_E_INVALID;
  }
  const hapod_precision prec = P->opts.prec;
  const int eb = elem_bytes(prec);
  const int64_t n = P->rows[a];
  const double eps = P->eps[a];
  const bool root = (a == P->root);
  if (m < 0 || lds < std::max<int64_t>(n, 1) || ldo < std::max<int64_t>(n, 1) || (m > 0 && (!S || !out))) {
    set_error("hapod_plan_node_pod: bad sizes or NULL pointer");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  *rank = 0;
  if (eps == 0.0) {  // POD(S, 0) = {(1, s)}
    if (m > 0) HAPOD_HIP(hipMemcpy2DAsync(out, ldo * eb, S, lds * eb, n * eb, m, hipMemcpyDeviceToDevice, stream));
    HAPOD_HIP(hipStreamSynchronize(stream));
    *rank = m;
    if (sigma)
      for (int64_t i = 0; i < m; ++i) sigma[i] = 1.0;
    return HAPOD_OK;
  }
  if (m == 0) return HAPOD_OK;
  auto to_caller = [&](int64_t, double** o, int64_t* ocs, int64_t* obs) {
    *o = (double*)out;
    *ocs = ldo;
    *obs = kRowBlock;
    return HAPOD_OK;
  };
  std::vector<double> sg;
  hapod_status st = HAPOD_OK;
  const int64_t ell = P->opts.sketch_cols;
  if (ell > 0 && m >= 2 * ell && n >= ell) {
    // the route, sketch width and seed a run gives this node
    const uint64_t seed = 0x6a09e667f3bcc909ull ^ ((uint64_t)a * 0x9e3779b97f4a7c15ull);
    std::vector<const void*> cols = column_table(S, lds, m, 8);
    std::vector<int64_t> rbs((size_t)m, kRowBlock), rows((size_t)m, n);
    st = sketch_pod_core(P->pool, n, m, cols, rbs, rows, ell, seed, P->opts.sketch_kind, eps, !root, to_caller, sg,
                         rank, nullptr, stream);
  } else if (P->opts.qr_pod && m <= kQrMaxM && m <= n) {
    st = qr_pod_core(P->pool, n, m, (double*)const_cast<void*>(S), lds, false, false, eps, !root, to_caller, sg, rank,
                     nullptr, nullptr, stream);
  } else {
    std::vector<PodJob> jobs(1);
    jobs[0].cols = column_table(S, lds, m, eb);
    jobs[0].rbs.assign((size_t)m, kRowBlock);
    jobs[0].crows.assign((size_t)m, n);
    jobs[0].n = n;
    jobs[0].m = m;
    jobs[0].eps = eps;
    jobs[0].root = root;
    jobs[0].out = out;
    jobs[0].ocs = ldo;
    jobs[0].obs = kRowBlock;
    const int jmax = P->opts.jacobi_max > 0 ? std::min<int>(P->opts.jacobi_max, kJacobiMax) : 0;
    st = run_pod_batch(prec, jobs, 0, 1, jmax, P->pool, stream, nullptr, nullptr, P->opts.autotune != 0);
    if (st == HAPOD_OK) {
      *rank = jobs[0].rank;
      sg = jobs[0].sigma;
    }
  }
  if (st == HAPOD_OK && sigma && *rank > 0) std::memcpy(sigma, sg.data(), sizeof(double) * *rank);
  return st;
}

hapod_status hapod_node_pod_qr(int64_t n, int64_t m, const double* S, int64_t lds, double eps, int32_t scaled,
                               double* out, int64_t ldo, double* sigma, int64_t* rank, int32_t* passes,
                               int32_t* sweeps, void* stream_) {
  if (n < 0 || m < 0 || !(eps >= 0.0) || !rank || lds < std::max<int64_t>(n, 1) || ldo < std::max<int64_t>(n, 1) ||
      (n > 0 && m > 0 && (!S || !out))) {
    set_error("hapod_node_pod_qr: bad argument");
    return HAPOD_E_INVALID;
  }
  if (m > kQrMaxM) {
    set_error("hapod_node_pod_qr: m above 512");
    return HAPOD_E_UNSUPPORTED;
  }
  if (m > n && eps > 0.0) {
    set_error("hapod_node_pod_qr: more columns than rows (no orthonormal Q of m columns)");
    return HAPOD_E_UNSUPPORTED;
  }
  hipStream_t stream = (hipStream_t)stream_;
  if (sweeps) *sweeps = 0;
  if (passes) *passes = 0;
  if (eps == 0.0) {  // POD(S, 0) = {(1, s)}
    if (n > 0 && m > 0)
      HAPOD_HIP(hipMemcpy2DAsync(out, ldo * 8, S, lds * 8, n * 8, m, hipMemcpyDeviceToDevice, stream));
    HAPOD_HIP(hipStreamSynchronize(stream));
    *rank = m;
    if (sigma)
      for (int64_t i = 0; i < m; ++i) sigma[i] = 1.0;
    return HAPOD_OK;
  }
  *rank = 0;
  if (m == 0 || n == 0) return HAPOD_OK;
  std::vector<double> sg;
  auto to_caller = [&](int64_t, double** o, int64_t* ocs, int64_t* obs) {
    *o = out;
    *ocs = ldo;
    *obs = kRowBlock;
    return HAPOD_OK;
  };
  hapod_status st = qr_pod_core(step_pool(), n, m, const_cast<double*>(S), lds, false, false, eps, scaled != 0, to_caller, sg,
                                rank, passes, sweeps, stream);
  if (st == HAPOD_OK && sigma && *rank > 0) std::memcpy(sigma, sg.data(), sizeof(double) * *rank);
  return st;
}

hapod_status hapod_node_pod_sketch(int64_t n, int64_t m, const double* S, int64_t lds, double eps, int32_t scaled,
                                   int64_t ell, uint64_t seed, int32_t kind, double* out, int64_t ldo, double* sigma,
                                   int64_t* rank, double* info7, void* stream_) {
  if (n < 0 || m < 0 || !(eps > 0.0) || !rank || lds < std::max<int64_t>(n, 1) || (m > 0 && n > 0 && (!S || !out)) ||
      ldo < std::max<int64_t>(n, 1)) {
    set_error("hapod_node_pod_sketch: bad sizes, eps <= 0 or NULL pointer");
    return HAPOD_E_INVALID;
  }
  if (ell < kGramTile || ell > kSketchMaxCols || ell % kGramTile != 0 || m < ell || n < ell) {
    set_error("hapod_node_pod_sketch: ell must be 128, 256, 384 or 512 and at most m and n");
    return HAPOD_E_UNSUPPORTED;
  }
  if (kind != 0 && kind != 1) {
    set_error("hapod_node_pod_sketch: kind must be 0 (sparse sign map, Gaussian fallback) or 1 (Gaussian)");
    return HAPOD_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_;
  *rank = 0;
  auto to_caller = [&](int64_t, double** o, int64_t* ocs, int64_t* obs) {
    *o = out;
    *ocs = ldo;
    *obs = kRowBlock;
    return HAPOD_OK;
  };
  std::vector<const void*> cols = column_table(S, lds, m, 8);
  std::vector<int64_t> rbs((size_t)m, kRowBlock), rows((size_t)m, n);
  std::vector<double> sg;
  SketchInfo si;
  hapod_status st = sketch_pod_core(step_pool(), n, m, cols, rbs, rows, ell, seed, kind, eps, scaled != 0, to_caller,
                                    sg, rank, &si, stream);
  if (info7) {
    const double v[7] = {si.residual, (double)si.passes_y, (double)si.passes_b, (double)si.sweeps,
                         (double)(si.ms[0] + si.ms[1] + si.ms[2] + si.ms[3] + si.ms[4] + si.ms[5]), (double)si.ell,
                         (double)si.kind};
    std::memcpy(info7, v, sizeof(v));
  }
  if (st == HAPOD_OK && sigma && *rank > 0) std::memcpy(sigma, sg.data(), sizeof(double) * *rank);
  return st;
}

}  // extern "C"
