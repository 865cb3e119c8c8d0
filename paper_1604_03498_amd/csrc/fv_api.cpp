// libfv host runtime: C ABI entry points, GMM constant precompute (double precision),
// per-stream workspaces, and the launch sequences of the encoder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "fv.h"
#include "fv_internal.h"


namespace {

thread_local int t_last_hip_error = 0;

// Serial numbers of loaded handles, starting at 1 (0 means "no handle" in a graph key).
std::atomic<uint64_t> g_next_serial{1};

constexpr unsigned kAllFlags =
    FV_X_DEVICE | FV_OUT_DEVICE | FV_NO_POWER_NORM | FV_NO_L2_NORM | FV_ASYNC | FV_THRESHOLD;
// flags that change what a captured sequence computes
constexpr unsigned kGraphFlags = FV_NO_POWER_NORM | FV_NO_L2_NORM | FV_THRESHOLD;

// The model's constants with this call's threshold setting.
fv::Consts call_consts(const fv_gmm* g, unsigned flags) {
  fv::Consts c = g->c;
  c.thresh = (flags & FV_THRESHOLD) ? 1 : 0;
  c.variant16 = g->fused16_variant;
  return c;
}

int hip_fail(hipError_t e) {
  t_last_hip_error = (int)e;
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FV_E_NOMEM : FV_E_DEVICE;
}

#define FV_HIP(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

// Makes `device` current for the lifetime of the guard and restores the caller's device.
class DeviceGuard {
 public:
  explicit DeviceGuard(int device) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    status_ = (prev_ == device) ? hipSuccess : hipSetDevice(device);
  }
  ~DeviceGuard() {
    if (prev_ >= 0 && status_ == hipSuccess) (void)hipSetDevice(prev_);
  }
  hipError_t status() const { return status_; }

 private:
  int prev_ = -1;
  hipError_t status_ = hipSuccess;
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

int device_cu_count(int device) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(device);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0)
    n = 256;
  cache[device] = n;
  return n;
}

// Device scratch (partials, tables, staging) and pinned host staging, cached per (device,
// stream).  Work on one stream is ordered, so reusing the buffers between calls is safe; a
// buffer is only replaced after the stream has drained.
// Everything a captured launch sequence bakes in: a replay is valid only for an equal key.
// Handles enter by serial number, not address: a handle loaded after another was freed may
// reuse its address, and a graph holds the old handle's device pointers.
struct GraphKey {
  int kind = 0;  // 0 = fv_encode, 1 = fv_encode_batch
  uint64_t gmm = 0;
  int precision = 0;
  unsigned flags = 0;
  int path = 0, P = 0;
  int64_t rows = 0;
  int B = 0, n_items = 0, n_groups = 0;
  const void* X = nullptr;
  const void* out = nullptr;
  const void* dev = nullptr;
  const void* pinned = nullptr;
  uint64_t pca = 0;  // 0: no projection
  int cap = 0;       // FV_MAX_GRID in force at capture (0: none)
  int grid = 0, variant = 0;  // the handle's batch_grid and fused16_variant tuning
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && gmm == o.gmm && precision == o.precision && flags == o.flags &&
           cap == o.cap && grid == o.grid && variant == o.variant &&
           path == o.path && P == o.P && rows == o.rows && B == o.B && n_items == o.n_items &&
           n_groups == o.n_groups && X == o.X && out == o.out && dev == o.dev &&
           pinned == o.pinned && pca == o.pca;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
};

// A capacity that holds `need`: unchanged if it does, else at least doubled (and >= lo).
int grow_cap(int cur, int need, int lo) {
  if (need <= cur) return cur;
  int64_t c = std::max<int64_t>({(int64_t)need, 2 * (int64_t)cur, (int64_t)lo});
  return (int)std::min<int64_t>(c, (int64_t)1 << 30);
}
int64_t grow_cap64(int64_t cur, int64_t need, int64_t lo) {
  if (need <= cur) return cur;
  return std::max<int64_t>({need, 2 * cur, lo});
}

struct Workspace {
  std::mutex mu;
  char* dev = nullptr;
  size_t dev_cap = 0;
  // Pinned staging of the batch tables: two halves of pin_cap bytes, filled by alternate calls,
  // so that a call waits only for the sequence before the previous one to have read its half
  // (the host builds the next batch's tables while the current one runs).
  char* pinned = nullptr;
  size_t pin_cap = 0;
  int pin_half = 0;                             // the half the next call fills
  hipEvent_t pin_done[2] = {nullptr, nullptr};  // end of the last sequence that read each half
  bool pin_pending[2] = {false, false};
  std::vector<GraphEntry> graphs;  // most recent last
  fv::BatchCaps caps;  // of the batched sequence (grow by doubling, or set by batch_reserve)
  int64_t captures = 0, replays = 0;  // graph captures and replays on this stream
};

std::atomic<int64_t> g_graph_captures{0}, g_graph_replays{0};

constexpr size_t kMaxGraphs = 16;

void drop_graphs(Workspace* ws) {
  for (auto& g : ws->graphs) (void)hipGraphExecDestroy(g.exec);
  ws->graphs.clear();
}

// Graph replay of launch sequences: on for device-resident inputs and outputs on a non-null
// stream, unless FV_GRAPH=0 or kernel timing is on.
bool graphs_enabled() {
  const char* e = std::getenv("FV_GRAPH");
  return !(e && e[0] == '0');
}

// Runs `enqueue` on stream s directly, or replays (capturing on first use) a graph cached
// under `key` in the workspace.
template <class F>
int run_sequence(Workspace* ws, const GraphKey& key, bool use_graph, hipStream_t s, F&& enqueue) {
  if (!use_graph) return enqueue();
  for (size_t i = 0; i < ws->graphs.size(); ++i)
    if (ws->graphs[i].key == key) {
      GraphEntry e = ws->graphs[i];
      ws->graphs.erase(ws->graphs.begin() + (long)i);
      ws->graphs.push_back(e);
      FV_HIP(hipGraphLaunch(e.exec, s));
      ++ws->replays;
      g_graph_replays.fetch_add(1, std::memory_order_relaxed);
      return FV_OK;
    }
  FV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue();
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (rc != FV_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec);
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(ei);
  if (ws->graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(ws->graphs.front().exec);
    ws->graphs.erase(ws->graphs.begin());
  }
  ws->graphs.push_back(GraphEntry{key, ex});
  ++ws->captures;
  g_graph_captures.fetch_add(1, std::memory_order_relaxed);
  FV_HIP(hipGraphLaunch(ex, s));
  return FV_OK;
}

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace* workspace_for(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto& p = g_ws[{device, s}];
  if (!p) p.reset(new (std::nothrow) Workspace());
  return p.get();
}

int ensure_dev(Workspace* ws, size_t need, hipStream_t s) {
  if (need <= ws->dev_cap) return FV_OK;
  if (ws->dev) {
    FV_HIP(hipStreamSynchronize(s));
    drop_graphs(ws);
    FV_HIP(hipFree(ws->dev));
    ws->dev = nullptr;
    ws->dev_cap = 0;
  }
  size_t cap = std::max(need, (size_t)(1u << 20));
  cap = align256(cap + cap / 4);
  FV_HIP(hipMalloc(&ws->dev, cap));
  ws->dev_cap = cap;
  return FV_OK;
}

int ensure_pinned(Workspace* ws, size_t need) {
  if (need > ws->pin_cap && ws->pinned) {
    for (int h = 0; h < 2; ++h)
      if (ws->pin_pending[h]) {
        FV_HIP(hipEventSynchronize(ws->pin_done[h]));
        ws->pin_pending[h] = false;
      }
    drop_graphs(ws);
    FV_HIP(hipHostFree(ws->pinned));
    ws->pinned = nullptr;
    ws->pin_cap = 0;
  }
  if (!ws->pinned) {
    const size_t cap = align256(std::max(need, (size_t)(64u << 10)) * 2);
    FV_HIP(hipHostMalloc(&ws->pinned, 2 * cap, hipHostMallocDefault));
    ws->pin_cap = cap;
  }
  const int h = ws->pin_half;
  if (ws->pin_pending[h]) {
    FV_HIP(hipEventSynchronize(ws->pin_done[h]));
    ws->pin_pending[h] = false;
  }
  if (!ws->pin_done[h]) FV_HIP(hipEventCreateWithFlags(&ws->pin_done[h], hipEventDisableTiming));
  return FV_OK;
}

bool finite_f(float v) { return std::isfinite(v); }

// Round-to-nearest-even conversions for the operand fragments (inputs are finite).
uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t f16_bits(_Float16 h) {
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

// ---- precision dispatch of the statistics kernels
fv::Frags16 frags(const fv::Consts& c, int precision) {
  switch (precision) {
    case FV_PREC_BF16_SPLIT: return fv::Frags16{c.Abf_hi, c.Abf_lo};
    case FV_PREC_FP16_SPLIT: return fv::Frags16{c.Ah_hi, c.Ah_lo};
    case FV_PREC_BF16: return fv::Frags16{c.Abf_hi, nullptr};
    default: return fv::Frags16{nullptr, nullptr};
  }
}

hipError_t run_stats(const fv::Consts& c, int prec, const float* X, bool vec_ok, int64_t N, int P,
                     const fv::Item* items, int n_items, int grid, float* partials, hipStream_t s) {
  const fv::Frags16 fr = frags(c, prec);
  switch (prec) {
    case FV_PREC_FP32: return fv::launch_stats(c, 0, X, vec_ok, N, P, items, n_items, grid, partials, s);
    case FV_PREC_BF16_SPLIT: return fv::launch_stats16_bf16s(c, fr, X, vec_ok, N, P, items, n_items, grid, partials, s);
    case FV_PREC_FP16_SPLIT: return fv::launch_stats16_f16s(c, fr, X, vec_ok, N, P, items, n_items, grid, partials, s);
    default: return fv::launch_stats16_bf16(c, fr, X, vec_ok, N, P, items, n_items, grid, partials, s);
  }
}

hipError_t run_lse(const fv::Consts& c, int prec, const float* X, bool vec_ok, int64_t N,
                   int n_tiles, int grid, float2* lse, int64_t stride, hipStream_t s,
                   float* gout = nullptr, int64_t gstride = 0) {
  const fv::Frags16 fr = frags(c, prec);
  switch (prec) {
    case FV_PREC_FP32: return fv::launch_lse(c, 0, X, vec_ok, N, nullptr, n_tiles, grid, lse, stride, s, gout, gstride);
    case FV_PREC_BF16_SPLIT: return fv::launch_lse16_bf16s(c, fr, X, vec_ok, N, nullptr, n_tiles, grid, lse, stride, s);
    case FV_PREC_FP16_SPLIT: return fv::launch_lse16_f16s(c, fr, X, vec_ok, N, nullptr, n_tiles, grid, lse, stride, s);
    default: return fv::launch_lse16_bf16(c, fr, X, vec_ok, N, nullptr, n_tiles, grid, lse, stride, s);
  }
}

hipError_t run_sliced(const fv::Consts& c, int prec, const float* X, bool vec_ok, int64_t N, int P,
                      const fv::Item* items, int n_items, int grid, const float2* lse,
                      int64_t stride, float* partials, hipStream_t s, const float* gin = nullptr,
                      int64_t gstride = 0) {
  const fv::Frags16 fr = frags(c, prec);
  switch (prec) {
    case FV_PREC_FP32: return fv::launch_sliced(c, 0, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s, gin, gstride);
    case FV_PREC_BF16_SPLIT: return fv::launch_sliced16_bf16s(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
    case FV_PREC_FP16_SPLIT: return fv::launch_sliced16_f16s(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
    default: return fv::launch_sliced16_bf16(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
  }
}

hipError_t run_normext(const fv::Consts& c, int prec, const float* X, bool vec_ok, int64_t N, int P,
                       const fv::Item* items, int n_items, int grid, const float2* lse,
                       int64_t stride, float* partials, hipStream_t s) {
  const fv::Frags16 fr = frags(c, prec);
  switch (prec) {
    case FV_PREC_FP32: return fv::launch_normext(c, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
    case FV_PREC_BF16_SPLIT: return fv::launch_normext16_bf16s(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
    case FV_PREC_FP16_SPLIT: return fv::launch_normext16_f16s(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
    default: return fv::launch_normext16_bf16(c, fr, X, vec_ok, N, P, items, n_items, grid, lse, stride, partials, s);
  }
}

// Component groups per chunk of the group-wise second pass (its workgroups have Wg waves, or 4
// when Wg = 8 and DP > 64; the 16-bit forms' pipelined kernel covers 256 components).
int normext_groups(const fv::Consts& c, int precision) {
  if (precision != FV_PREC_FP32 && fv::normext16_pipelined(c)) return c.Kp / (8 * fv::kCompsPerWave);
  const int w = (c.DP > 64 && c.Wg == 8) ? 4 : c.Wg;
  return c.Kp / (fv::kCompsPerWave * w);
}

// Rows one second-pass workgroup consumes per round of its waves (32-row tiles).
int sliced_round(const fv::Consts& c, int prec) {
  switch (prec) {
    case FV_PREC_FP32: return fv::sliced_rows_per_wave_round(c.DP);
    case FV_PREC_BF16_SPLIT: return fv::kTile * fv::sliced16_waves_bf16s(c.DP);
    case FV_PREC_FP16_SPLIT: return fv::kTile * fv::sliced16_waves_f16s(c.DP);
    default: return fv::kTile * fv::sliced16_waves_bf16(c.DP);
  }
}

enum class Path { kFused, kSplit };

// The FP32 two-pass path's posterior hand-over (first pass writes e and the row scales, second
// pass reads them): on unless FV_SPLIT_GAMMA=0 (tests and measurements).  Its buffer,
// (Kp + Kp / 32) x N floats, is used up to this size; larger frames recompute the E-step.
constexpr size_t kMaxGammaBytes = (size_t)256 << 20;
bool split_gamma_enabled() {
  const char* e = std::getenv("FV_SPLIT_GAMMA");
  return !(e && e[0] == '0');
}

// Persistent-grid cap for tests and measurements: FV_MAX_GRID=n limits the first grid
// dimension of every statistics launch to n workgroups, so each workgroup loops over several
// work items (the kernels are grid-stride over their items; results do not depend on it).
int grid_cap(int g) {
  const char* e = std::getenv("FV_MAX_GRID");
  if (!e) return g;
  const int x = std::atoi(e);
  return x >= 1 ? std::min(g, x) : g;
}

// FV_FUSED16 (measurements): w, t or p forces the 16-bit fused kernel variant 1, 2 or 3.
int fused16_env() {
  const char* e = std::getenv("FV_FUSED16");
  if (!e) return 0;
  return e[0] == 'w' ? 1 : e[0] == 't' ? 2 : e[0] == 'p' ? 3 : 0;
}

// Path override for tests and measurements: FV_PATH=fused|split (default: automatic).
int path_override() {
  const char* e = std::getenv("FV_PATH");
  if (!e) return 0;
  if (std::strcmp(e, "fused") == 0) return 1;
  if (std::strcmp(e, "split") == 0) return 2;
  return 0;
}

// Workgroups of the fused kernel (or of the first pass) that fit on the device at once:
// one 8-wave workgroup per CU at 256 components (register bound), more for fewer waves.
int resident_fused(int device, int Wg) { return device_cu_count(device) * std::max(1, 8 / Wg); }

// Above DP = 64 the 8-wave FP32 fused kernel spills registers, and the two-pass path (whose
// group-wise second pass runs 4 waves there) is as fast or faster: 32 frames at K = 256 took
// 1.14 against 1.15 ms at D = 80 and 1.45 against 1.85 ms at D = 96.  The 16-bit forms keep
// the fused kernel (0.35 against 0.45 ms at D = 80).
bool fused_spills(const fv_gmm* g, int precision) {
  return precision == FV_PREC_FP32 && g->c.DP > 64 && g->c.Wg == fv::kMaxWaves;
}

// Single frame: the fused kernel needs several 32-row tiles per resident workgroup to amortise
// its per-chunk partial write; below that the two-pass path (more, smaller workgroups and
// fewer partial slots) is used.  More than 256 components always take the two-pass path.
Path choose_single(const fv_gmm* g, int64_t N, int precision) {
  const fv::Consts& c = g->c;
  if (c.Kp > fv::kFusedMaxK) return Path::kSplit;
  const int o = path_override();
  if (o == 1) return Path::kFused;
  if (o == 2) return Path::kSplit;
  if (fused_spills(g, precision) && g->single_split_below == 0) return Path::kSplit;
  const int64_t below = g->single_split_below > 0
                            ? g->single_split_below
                            : (int64_t)4 * fv::kTile * resident_fused(g->device, c.Wg);
  return N < below ? Path::kSplit : Path::kFused;
}

Path choose_batch(const fv_gmm* g, int precision) {
  if (g->c.Kp > fv::kFusedMaxK) return Path::kSplit;
  const int o = path_override();
  if (o == 1) return Path::kFused;
  if (o == 2) return Path::kSplit;
  if (g->batch_path != 0) return g->batch_path == 2 ? Path::kSplit : Path::kFused;
  return fused_spills(g, precision) ? Path::kSplit : Path::kFused;
}

// Chunk length of the fused kernel for a single frame: enough items to give every resident
// workgroup work, in whole tiles.
int fused_single_chunk(int64_t N, int device, int Wg) {
  const int64_t target = resident_fused(device, Wg);
  const int64_t tiles = (N + fv::kTile - 1) / fv::kTile;
  const int64_t per = std::max<int64_t>(1, (tiles + target - 1) / target);
  return (int)std::min<int64_t>(per * fv::kTile, (int64_t)1 << 20);
}

// Grid width of the second pass.  Workgroups go to the eight XCDs (each with its own L2) in
// round-robin order of their linear index x + y * gridDim.x; with gridDim.x a multiple of 8
// every component slice y of chunk x runs on the same XCD, so the chunk's rows are fetched
// from HBM once and then hit that XCD's L2.  Workgroups past the last chunk exit at once.
int xcd_grid(int n) { return (n + 7) / 8 * 8; }

// Chunk length of the second pass for a single frame: about one workgroup per CU over all
// (chunk, slice) pairs, in whole rounds of the workgroup's 32-row tiles.  Measured on the
// 8,000-row frame (K = 256, D = 64, FP32, four-wave workgroups): 41 us at one workgroup per
// CU, 42 us at two, 46 and 51 us at 3/4 and 1/2.
int split_single_chunk(int64_t N, int device, int slices, int round) {
  const int64_t target_chunks =
      std::max<int64_t>(1, ((int64_t)device_cu_count(device) + slices - 1) / slices);
  const int64_t per = (N + target_chunks - 1) / target_chunks;
  const int64_t P = std::max<int64_t>(round, (per + round - 1) / round * round);
  return (int)std::min<int64_t>(P, (int64_t)1 << 20);
}

// Chunk length of the group-wise second pass for a single frame: about one workgroup per CU
// over all (chunk, component group) pairs, in whole tiles.
int normext_single_chunk(int64_t N, int device, int groups) {
  const int64_t target = std::max<int64_t>(1, (device_cu_count(device) + groups - 1) / groups);
  const int64_t tiles = (N + fv::kTile - 1) / fv::kTile;
  const int64_t per = std::max<int64_t>(1, (tiles + target - 1) / target);
  return (int)std::min<int64_t>(per * fv::kTile, (int64_t)1 << 20);
}

// Frame-relative chunk length of the batched path (a multiple of 128 rows): FV_BATCH_CHUNK
// (test override), else the handle's tuning, else 1024.
int batch_chunk(const fv_gmm* g) {
  if (const char* e = std::getenv("FV_BATCH_CHUNK")) {
    const int x = std::atoi(e);
    if (x >= 128) return (x / 128) * 128;
  }
  if (g->batch_chunk >= 128) return (g->batch_chunk / 128) * 128;
  return 1024;
}

// ---- optional kernel timing: event pairs recorded around launches on the launch stream
struct TimingState {
  std::mutex mu;
  bool enabled = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];
  std::vector<hipEvent_t> pool;
  double total_ms[3] = {0.0, 0.0, 0.0};
  int64_t launches[3] = {0, 0, 0};
};
TimingState g_timing;

hipEvent_t timing_event() {
  hipEvent_t e = nullptr;
  if (!g_timing.pool.empty()) {
    e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

bool timing_enabled() {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  return g_timing.enabled;
}

// Records a start event when timing is on; returns it (or null).
hipEvent_t timing_begin(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (!g_timing.enabled) return nullptr;
  hipEvent_t e = timing_event();
  if (e && hipEventRecord(e, s) != hipSuccess) {
    g_timing.pool.push_back(e);
    return nullptr;
  }
  return e;
}

void timing_end(hipEvent_t start, int which, hipStream_t s) {
  if (!start) return;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  hipEvent_t e = timing_event();
  if (!e || hipEventRecord(e, s) != hipSuccess) {
    g_timing.pool.push_back(start);
    if (e) g_timing.pool.push_back(e);
    return;
  }
  g_timing.pending[which].push_back({start, e});
}

// Workgroups of the projection kernel: two per CU (register bound), grid-stride over tiles of
// at least 32 rows (extra workgroups exit at once).
int project_grid(int device, int64_t N) {
  const int64_t tiles = (N + fv::kTile - 1) / fv::kTile;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)device_cu_count(device) * 2));
}

// Byte layout of a stream's batch workspace for capacities `cp`: partial slots, finalize
// norm parts, first-pass normalisers (two-pass path), the work table (Counts record, frames,
// items, item order), staging of host X and host out, and the projected rows.
struct BatchLayout {
  size_t part = 0, norm = 0, lse = 0, cnt = 0, frames = 0, items = 0, order = 0;
  size_t x = 0, out = 0, y = 0;
  size_t tab() const { return cnt + frames + items + order; }
  size_t total() const { return part + norm + lse + tab() + x + out + y; }
};

BatchLayout batch_layout(const fv::Consts& c, Path path, const fv::BatchCaps& cp, int Din,
                         unsigned flags, bool pca) {
  BatchLayout l;
  const size_t out_len = (size_t)2 * c.K * c.D;
  l.part = align256((size_t)cp.items * fv::slot_floats(c) * 4);
  l.norm = align256((size_t)cp.B * fv::finalize_blocks(c) * 8);
  l.lse = (path == Path::kSplit) ? align256((size_t)fv::lse_groups(c) * cp.rows * 8) : 0;
  l.cnt = align256(sizeof(fv::Counts));
  l.frames = align256((size_t)cp.B * sizeof(fv::Frame));
  l.items = align256((size_t)cp.items * sizeof(fv::Item));
  l.order = align256((size_t)cp.items * sizeof(int32_t));
  l.x = (flags & FV_X_DEVICE) ? 0 : align256((size_t)cp.rows * Din * 4);
  l.out = (flags & FV_OUT_DEVICE) ? 0 : align256((size_t)cp.B * out_len * 4);
  l.y = pca ? align256((size_t)cp.rows * c.D * 4) : 0;
  return l;
}

}  // namespace

namespace fv {
void stream_graph_counts(int device, hipStream_t s, int64_t* captures, int64_t* replays) {
  Workspace* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({device, s});
    if (it != g_ws.end()) ws = it->second.get();
  }
  int64_t c = 0, r = 0;
  if (ws) {
    std::lock_guard<std::mutex> lk(ws->mu);
    c = ws->captures;
    r = ws->replays;
  }
  if (captures) *captures = c;
  if (replays) *replays = r;
}

BatchCaps batch_need(const fv_gmm* g, const int64_t* sizes, int B) {
  const int P = batch_chunk(g);
  BatchCaps n;
  n.B = B;
  int64_t items = 0, groups = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t ni = (sizes[b] + P - 1) / P;
    n.rows += sizes[b];
    items += ni;
    groups += (ni + kGroupItems - 1) / kGroupItems;
  }
  n.items = (int)std::min<int64_t>(items, (int64_t)1 << 30);
  n.groups = (int)std::min<int64_t>(groups, (int64_t)1 << 30);
  return n;
}

size_t batch_caps_bytes(const fv_gmm* g, int precision, const BatchCaps& caps) {
  return batch_layout(g->c, choose_batch(g, precision), caps, g->D, FV_X_DEVICE | FV_OUT_DEVICE,
                      false)
      .total();
}

int batch_reserve(const fv_gmm* g, int precision, hipStream_t s, const BatchCaps& caps,
                  size_t* bytes) {
  if (!g || !bytes) return FV_E_INVAL;
  DeviceGuard dg(g->device);
  if (dg.status() != hipSuccess) return hip_fail(dg.status());
  Workspace* ws = workspace_for(g->device, s);
  if (!ws) return FV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ws->mu);
  const size_t need = batch_caps_bytes(g, precision, caps);
  if (need != ws->dev_cap) {
    if (ws->dev) {
      FV_HIP(hipStreamSynchronize(s));
      drop_graphs(ws);
      FV_HIP(hipFree(ws->dev));
      ws->dev = nullptr;
      ws->dev_cap = 0;
    }
    if (need > 0) {
      FV_HIP(hipMalloc(&ws->dev, need));
      ws->dev_cap = need;
    }
  }
  ws->caps = caps;
  *bytes = ws->dev_cap;
  return FV_OK;
}
}  // namespace fv

extern "C" {

int fv_kernel_timing(int enable) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  for (int w = 0; w < 3; ++w) {
    for (auto& pr : g_timing.pending[w]) {
      (void)hipEventSynchronize(pr.second);
      g_timing.pool.push_back(pr.first);
      g_timing.pool.push_back(pr.second);
    }
    g_timing.pending[w].clear();
    g_timing.total_ms[w] = 0.0;
    g_timing.launches[w] = 0;
  }
  g_timing.enabled = enable != 0;
  return FV_OK;
}

int fv_kernel_timing_read(int which, double* total_ms, int64_t* launches) {
  if (which < 0 || which > 2) return FV_E_INVAL;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  for (auto& pr : g_timing.pending[which]) {
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e);
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e);
    g_timing.total_ms[which] += ms;
    g_timing.launches[which] += 1;
    g_timing.pool.push_back(pr.first);
    g_timing.pool.push_back(pr.second);
  }
  g_timing.pending[which].clear();
  if (total_ms) *total_ms = g_timing.total_ms[which];
  if (launches) *launches = g_timing.launches[which];
  return FV_OK;
}

void fv_limits(int* max_K, int* max_D) {
  if (max_K) *max_K = fv::kMaxK;
  if (max_D) *max_D = fv::kMaxD;
}

const char* fv_strerror(int code) {
  switch (code) {
    case FV_OK: return "ok";
    case FV_PENDING: return "pending";
    case FV_E_INVAL: return "invalid argument";
    case FV_E_NOMEM: return "out of memory";
    case FV_E_DEVICE: return "device (HIP runtime) error";
    case FV_E_BUDGET: return "request exceeds the device-memory budget";
    case FV_E_AGAIN: return "queue full, try again";
    case FV_E_NOTFOUND: return "unknown ticket";
    case FV_E_TIMEOUT: return "deadline exceeded";
    case FV_E_UNSUPPORTED: return "unsupported size or form";
    default: return "unknown status";
  }
}

int fv_last_device_error(void) { return t_last_hip_error; }

int fv_graph_counters(int64_t* captures, int64_t* replays) {
  if (captures) *captures = g_graph_captures.load(std::memory_order_relaxed);
  if (replays) *replays = g_graph_replays.load(std::memory_order_relaxed);
  return FV_OK;
}

int fv_stream_release(int device, void* hip_stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  std::unique_ptr<Workspace> ws;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({device, s});
    if (it != g_ws.end()) {
      ws = std::move(it->second);
      g_ws.erase(it);
    }
  }
  const bool front = fv::dsift_in_use(device, s);
  if (!ws && !front) return FV_OK;  // a pair never used: no device call at all
  DeviceGuard g(device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  const int rc_front = fv::dsift_release(device, s);
  if (!ws) return rc_front;
  std::lock_guard<std::mutex> lk(ws->mu);
  int rc = FV_OK;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) rc = hip_fail(e);
  drop_graphs(ws.get());
  if (ws->dev && (e = hipFree(ws->dev)) != hipSuccess) rc = hip_fail(e);
  if (ws->pinned && (e = hipHostFree(ws->pinned)) != hipSuccess) rc = hip_fail(e);
  for (hipEvent_t& ev : ws->pin_done)
    if (ev) (void)hipEventDestroy(ev);
  ws->dev = ws->pinned = nullptr;
  return rc != FV_OK ? rc : rc_front;
}

int fv_gmm_load(int K, int D, const float* priors, const float* means, const float* variances,
                int device, fv_gmm** out) {
  if (!out) return FV_E_INVAL;
  *out = nullptr;
  if (K < 1 || D < 1 || !priors || !means || !variances) return FV_E_INVAL;
  for (int k = 0; k < K; ++k)
    if (!finite_f(priors[k]) || !(priors[k] > 0.f)) return FV_E_INVAL;
  const size_t KD = (size_t)K * D;
  for (size_t i = 0; i < KD; ++i) {
    if (!finite_f(means[i])) return FV_E_INVAL;
    if (!finite_f(variances[i]) || !(variances[i] > 0.f)) return FV_E_INVAL;
  }
  if (K > fv::kMaxK || D > fv::kMaxD) return FV_E_UNSUPPORTED;
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess) return hip_fail(de);
  if (device < 0 || device >= ndev) return FV_E_INVAL;

  fv::Consts c{};
  c.K = K;
  c.D = D;
  if (K <= fv::kFusedMaxK) {
    c.Wg = 1;
    while (c.Wg * fv::kCompsPerWave < K) c.Wg *= 2;
    c.Kp = c.Wg * fv::kCompsPerWave;
  } else {
    c.Wg = fv::kMaxWaves;
    const int grp = fv::kMaxWaves * fv::kCompsPerWave;
    c.Kp = (K + grp - 1) / grp * grp;
  }
  c.DP = ((D + 15) / 16) * 16;
  const int Kp = c.Kp, DP = c.DP;

  // ---- precompute in double (the paper's "compute sqrt(sigma^-1)" step, widened to every
  // per-model constant the kernels need)
  const double LOG2E = 1.4426950408889634073599246810019;
  std::vector<float> A((size_t)2 * DP * Kp, 0.f), cc((size_t)Kp, -1e30f);
  const size_t nfrag = (size_t)2 * DP * Kp;  // same element count as A, fragment order
  std::vector<uint16_t> abh(nfrag, 0), abl(nfrag, 0), ahh(nfrag, 0), ahl(nfrag, 0);
  bool f16_fits = true;
  std::vector<double> mu64(KD), isd64(KD), ivar64(KD), cu64(K), cv64(K);
  // model centre m0 = sum_k w_k mu_k / sum_k w_k, rounded to float: the kernels encode x - m0
  // against the means mu - m0 (exact in double), which leaves the Fisher vector unchanged and
  // keeps x, x^2, the operand entries and the raw moments small for data far from the origin
  std::vector<float> cen((size_t)DP, 0.f);
  {
    double wsum = 0.0;
    for (int k = 0; k < K; ++k) wsum += (double)priors[k];
    for (int d = 0; d < D; ++d) {
      double a = 0.0;
      for (int k = 0; k < K; ++k) a += (double)priors[k] * (double)means[(size_t)k * D + d];
      cen[d] = (float)(a / wsum);
    }
  }
  for (int k = 0; k < K; ++k) {
    double logdet = 0.0, quad = 0.0;
    for (int d = 0; d < D; ++d) {
      const double m = (double)means[(size_t)k * D + d] - (double)cen[d];
      const double v = variances[(size_t)k * D + d];
      const double iv = 1.0 / v;
      A[(size_t)d * Kp + k] = (float)(m * iv * LOG2E);
      A[(size_t)(DP + d) * Kp + k] = (float)(-0.5 * iv * LOG2E);
      logdet += std::log(v);
      quad += m * m * iv;
      mu64[(size_t)k * D + d] = m;
      isd64[(size_t)k * D + d] = 1.0 / std::sqrt(v);
      ivar64[(size_t)k * D + d] = iv;
    }
    const double w = priors[k];
    cc[k] = (float)((std::log(w) - 0.5 * logdet - 0.5 * quad) * LOG2E);
    cu64[k] = 1.0 / std::sqrt(w);
    cv64[k] = 1.0 / std::sqrt(2.0 * w);
  }

  // 16-bit hi/lo operand fragments: fragment (s, h, comp) = A[16s + 8h + e][comp], e = 0..7
  for (int st = 0; st < 2 * DP / 16; ++st)
    for (int hh = 0; hh < 2; ++hh)
      for (int k = 0; k < Kp; ++k)
        for (int e = 0; e < 8; ++e) {
          const float v = A[(size_t)(16 * st + 8 * hh + e) * Kp + k];
          const size_t o = (((size_t)st * 2 + hh) * Kp + k) * 8 + e;
          const uint16_t bh = bf16_rne(v);
          abh[o] = bh;
          abl[o] = bf16_rne(v - bf16_to_f32(bh));
          const _Float16 fh = (_Float16)v;
          f16_fits = f16_fits && std::isfinite((float)fh);
          ahh[o] = f16_bits(fh);
          ahl[o] = f16_bits((_Float16)(v - (float)fh));
        }

  // FP32 operand in fragment order (see Consts::A32)
  std::vector<float> Af(A.size(), 0.f);
  for (int cb = 0; cb < Kp / fv::kCompsPerWave; ++cb)
    for (int gq = 0; gq < DP / 4; ++gq)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 4; ++e)
          Af[(((size_t)cb * (DP / 4) + gq) * 64 + l) * 4 + e] =
              A[(size_t)(4 * gq + e + DP * (l >> 5)) * Kp + cb * fv::kCompsPerWave + (l & 31)];

  // ---- one device block: A32 | c32 | 4 x 16-bit operand fragments | doubles
  const size_t nA = A.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t oA = take(nA * 4), oc = take((size_t)Kp * 4), oCen = take((size_t)DP * 4);
  const size_t oBH = take(nfrag * 2), oBL = take(nfrag * 2), oHH = take(nfrag * 2), oHL = take(nfrag * 2);
  const size_t oMu = take(KD * 8), oIsd = take(KD * 8), oIvar = take(KD * 8);
  const size_t oCu = take((size_t)K * 8), oCv = take((size_t)K * 8);
  const size_t total = off;

  DeviceGuard g(device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  std::unique_ptr<fv_gmm> h(new (std::nothrow) fv_gmm());
  if (!h) return FV_E_NOMEM;
  char* blk = nullptr;
  FV_HIP(hipMalloc(&blk, total));
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + oA, Af.data(), nA * 4);
  std::memcpy(host.data() + oc, cc.data(), (size_t)Kp * 4);
  std::memcpy(host.data() + oCen, cen.data(), (size_t)DP * 4);
  std::memcpy(host.data() + oBH, abh.data(), nfrag * 2);
  std::memcpy(host.data() + oBL, abl.data(), nfrag * 2);
  std::memcpy(host.data() + oHH, ahh.data(), nfrag * 2);
  std::memcpy(host.data() + oHL, ahl.data(), nfrag * 2);
  std::memcpy(host.data() + oMu, mu64.data(), KD * 8);
  std::memcpy(host.data() + oIsd, isd64.data(), KD * 8);
  std::memcpy(host.data() + oIvar, ivar64.data(), KD * 8);
  std::memcpy(host.data() + oCu, cu64.data(), (size_t)K * 8);
  std::memcpy(host.data() + oCv, cv64.data(), (size_t)K * 8);
  hipError_t e = hipMemcpy(blk, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(blk);
    return hip_fail(e);
  }
  c.A32 = reinterpret_cast<const float*>(blk + oA);
  c.c32 = reinterpret_cast<const float*>(blk + oc);
  c.cen = reinterpret_cast<const float*>(blk + oCen);
  c.Abf_hi = reinterpret_cast<const uint16_t*>(blk + oBH);
  c.Abf_lo = reinterpret_cast<const uint16_t*>(blk + oBL);
  c.Ah_hi = reinterpret_cast<const uint16_t*>(blk + oHH);
  c.Ah_lo = reinterpret_cast<const uint16_t*>(blk + oHL);
  c.mu64 = reinterpret_cast<const double*>(blk + oMu);
  c.isd64 = reinterpret_cast<const double*>(blk + oIsd);
  c.ivar64 = reinterpret_cast<const double*>(blk + oIvar);
  c.cu64 = reinterpret_cast<const double*>(blk + oCu);
  c.cv64 = reinterpret_cast<const double*>(blk + oCv);
  h->K = K;
  h->D = D;
  h->device = device;
  h->serial = g_next_serial.fetch_add(1);
  h->f16_fits = f16_fits;
  h->c = c;
  h->dev_block = blk;
  *out = h.release();
  return FV_OK;
}

int fv_gmm_free(fv_gmm* gmm) {
  if (!gmm) return FV_OK;
  int rc = FV_OK;
  {
    DeviceGuard g(gmm->device);
    if (gmm->dev_block) {
      hipError_t e = hipFree(gmm->dev_block);
      if (e != hipSuccess) rc = hip_fail(e);
    }
  }
  delete gmm;
  return rc;
}

int fv_gmm_set_tuning(fv_gmm* gmm, const fv_tuning* t) {
  if (!gmm) return FV_E_INVAL;
  if (!t) {
    gmm->batch_chunk = 0;
    gmm->batch_path = 0;
    gmm->single_split_below = 0;
    gmm->batch_grid = 0;
    gmm->fused16_variant = 0;
    return FV_OK;
  }
  if (t->batch_chunk < 0 || (t->batch_chunk > 0 && t->batch_chunk < 128) || t->batch_path < 0 ||
      t->batch_path > 2 || t->single_split_below < 0 || t->batch_grid < 0 ||
      t->batch_grid > (1 << 20) || t->fused16_variant < 0 || t->fused16_variant > 3)
    return FV_E_INVAL;
  gmm->batch_chunk = t->batch_chunk;
  gmm->batch_path = t->batch_path;
  gmm->single_split_below = t->single_split_below;
  gmm->batch_grid = t->batch_grid;
  gmm->fused16_variant = t->fused16_variant;
  return FV_OK;
}

int fv_gmm_get_tuning(const fv_gmm* gmm, fv_tuning* t) {
  if (!gmm || !t) return FV_E_INVAL;
  t->batch_chunk = gmm->batch_chunk;
  t->batch_path = gmm->batch_path;
  t->single_split_below = gmm->single_split_below;
  t->batch_grid = gmm->batch_grid;
  t->fused16_variant = gmm->fused16_variant;
  return FV_OK;
}

int fv_gmm_info(const fv_gmm* gmm, int* K, int* D, int* device) {
  if (!gmm) return FV_E_INVAL;
  if (K) *K = gmm->K;
  if (D) *D = gmm->D;
  if (device) *device = gmm->device;
  return FV_OK;
}

}  // extern "C"

namespace {

// The single-frame launch plan: path, chunk length and the scratch each buffer takes.
struct SinglePlan {
  Path path = Path::kSplit;
  bool grouped = false, gam_path = false;
  int P = fv::kTile, n_items = 0, n_groups = 0, G = 1, nblk = 0;
  int64_t gstride = 0;
  size_t b_gam = 0, b_part = 0, b_norm = 0, b_lse = 0;
  size_t scratch() const { return b_part + b_norm + b_lse + b_gam; }
};

SinglePlan plan_single(const fv_gmm* gmm, const fv::Consts& c, int64_t N, int precision,
                       Path path, bool allow_gam) {
  SinglePlan p;
  p.path = path;
  const int slices = c.Kp / fv::kCompsPerWave;
  // the two-pass path's second pass: component-sliced workgroups up to 256 components (more
  // parallelism for one frame), whole component groups beyond
  p.grouped = c.Kp > fv::kFusedMaxK;
  if (N > 0)
    p.P = (path == Path::kFused) ? fused_single_chunk(N, gmm->device, c.Wg)
          : p.grouped            ? normext_single_chunk(N, gmm->device, normext_groups(c, precision))
                                 : split_single_chunk(N, gmm->device, slices, sliced_round(c, precision));
  p.n_items = N > 0 ? (int)((N + p.P - 1) / p.P) : 0;
  p.n_groups = (p.n_items + fv::kGroupItems - 1) / fv::kGroupItems;
  p.G = fv::lse_groups(c);
  p.nblk = fv::finalize_blocks(c);
  // FP32 two-pass with one component group: the first pass also writes the posterior factors
  // (e and the row scales) and the second pass reads them instead of recomputing the E-step
  p.gstride = (N + fv::kTile - 1) / fv::kTile * fv::kTile;
  const size_t gam_bytes = (size_t)(c.Kp + c.Kp / fv::kCompsPerWave) * p.gstride * 4;
  p.gam_path = allow_gam && path == Path::kSplit && !p.grouped && precision == FV_PREC_FP32 &&
               p.G == 1 && c.DP <= 64 && N > 0 && gam_bytes <= kMaxGammaBytes &&
               split_gamma_enabled();
  p.b_gam = p.gam_path ? align256(gam_bytes) : 0;
  p.b_part = align256((size_t)p.n_items * fv::slot_floats(c) * 4);
  p.b_norm = align256((size_t)p.nblk * 8);
  p.b_lse = (path == Path::kSplit) ? align256((size_t)p.G * N * 8) : 0;
  return p;
}

}  // namespace

extern "C" {

// fv_encode, with the projection prologue when pca is non-null (X then has pca->Din columns).
// With ext non-null (the allocation-free entry point) every intermediate lives in the ext_cap
// bytes at ext: X and out must be in device memory, nothing is allocated, no graph is captured
// and no timing event is recorded; the plan falls back to the two-pass path and then to the
// E-step recompute when the preferred one does not fit, and a frame that fits neither is
// refused with FV_E_UNSUPPORTED.
static int encode_impl(const fv_gmm* gmm, const fv_pca* pca, const float* X, int64_t N,
                       float* out, int precision, unsigned flags, void* hip_stream,
                       char* ext = nullptr, size_t ext_cap = 0) {
  if (!gmm || !out || N < 0 || (N > 0 && !X)) return FV_E_INVAL;
  if (const int fs = fv_form_status(gmm, precision)) return fs;
  if (flags & ~kAllFlags) return FV_E_INVAL;
  if (pca && (pca->D != gmm->D || pca->device != gmm->device)) return FV_E_INVAL;
  if (ext && (pca || !(flags & FV_X_DEVICE) || !(flags & FV_OUT_DEVICE))) return FV_E_INVAL;
  const fv::Consts c = call_consts(gmm, flags);
  const int Din = pca ? pca->Din : c.D;
  if (N > ((int64_t)1 << 40) / std::max(Din, c.D)) return FV_E_UNSUPPORTED;
  DeviceGuard g(gmm->device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Workspace* ws = nullptr;
  std::unique_lock<std::mutex> lk;
  if (!ext) {
    ws = workspace_for(gmm->device, s);
    if (!ws) return FV_E_NOMEM;
    lk = std::unique_lock<std::mutex>(ws->mu);
  }

  SinglePlan pl = plan_single(gmm, c, N, precision, choose_single(gmm, N, precision), true);
  if (ext && pl.scratch() > ext_cap && pl.path == Path::kFused)
    pl = plan_single(gmm, c, N, precision, Path::kSplit, true);
  if (ext && pl.scratch() > ext_cap && pl.gam_path)
    pl = plan_single(gmm, c, N, precision, pl.path, false);
  if (ext && pl.scratch() > ext_cap) return FV_E_UNSUPPORTED;
  const Path path = pl.path;
  const bool grouped = pl.grouped, gam_path = pl.gam_path;
  const int P = pl.P, n_items = pl.n_items, n_groups = pl.n_groups;
  const int64_t gstride = pl.gstride;
  const size_t out_len = (size_t)2 * c.K * c.D;
  const size_t b_gam = pl.b_gam, b_part = pl.b_part, b_norm = pl.b_norm, b_lse = pl.b_lse;
  const size_t b_x = (flags & FV_X_DEVICE) ? 0 : align256((size_t)N * Din * 4);
  const size_t b_out = (flags & FV_OUT_DEVICE) ? 0 : align256(out_len * 4);
  const size_t b_y = pca ? align256((size_t)N * c.D * 4) : 0;
  int rc = FV_OK;
  if (!ext) {
    rc = ensure_dev(ws, b_part + b_norm + b_lse + b_x + b_out + b_y + b_gam, s);
    if (rc) return rc;
  }
  char* base = ext ? ext : ws->dev;
  float* partials = reinterpret_cast<float*>(base);
  double* normpart = reinterpret_cast<double*>(base + b_part);
  float2* lse = reinterpret_cast<float2*>(base + b_part + b_norm);
  float* xdev = reinterpret_cast<float*>(base + b_part + b_norm + b_lse);
  float* odev = reinterpret_cast<float*>(base + b_part + b_norm + b_lse + b_x);
  float* ydev = reinterpret_cast<float*>(base + b_part + b_norm + b_lse + b_x + b_out);
  float* gam = gam_path ? reinterpret_cast<float*>(base + b_part + b_norm + b_lse + b_x + b_out + b_y)
                        : nullptr;

  const float* Xd = X;
  if (!(flags & FV_X_DEVICE) && N > 0) {
    FV_HIP(hipMemcpyAsync(xdev, X, (size_t)N * Din * 4, hipMemcpyHostToDevice, s));
    Xd = xdev;
  }
  if ((reinterpret_cast<uintptr_t>(Xd) & 3) != 0) return FV_E_INVAL;
  float* Od = (flags & FV_OUT_DEVICE) ? out : odev;
  // the encoder's input: the projected rows (library scratch) or X itself
  const float* Fx = pca ? ydev : Xd;
  const bool vec_ok = (c.D % 4 == 0) && ((reinterpret_cast<uintptr_t>(Fx) & 15) == 0);

  auto enqueue = [&]() -> int {
    if (pca && N > 0) {
      hipEvent_t tp = ext ? nullptr : timing_begin(s);
      FV_HIP(fv::launch_project(pca->p, Xd, N, ydev, project_grid(gmm->device, N), s, nullptr,
                                precision != FV_PREC_FP32));
      timing_end(tp, 2, s);
    }
    if (n_items > 0) {
      hipEvent_t t0 = ext ? nullptr : timing_begin(s);
      if (path == Path::kFused) {
        FV_HIP(run_stats(c, precision, Fx, vec_ok, N, P, nullptr, n_items, grid_cap(n_items), partials, s));
      } else {
        const int n_tiles = (int)((N + fv::kTile - 1) / fv::kTile);
        const int grid1 = grid_cap(std::min(n_tiles, resident_fused(gmm->device, c.Wg)));
        FV_HIP(run_lse(c, precision, Fx, vec_ok, N, n_tiles, grid1, lse, N, s, gam, gstride));
        const int grid2 = grid_cap(xcd_grid(n_items));
        if (grouped)
          FV_HIP(run_normext(c, precision, Fx, vec_ok, N, P, nullptr, n_items, grid2, lse, N,
                             partials, s));
        else
          FV_HIP(run_sliced(c, precision, Fx, vec_ok, N, P, nullptr, n_items, grid2, lse, N,
                            partials, s, gam, gstride));
      }
      timing_end(t0, 0, s);
    }
    fv::Frame single{N, 0, n_items, 0, n_groups};
    hipEvent_t t1 = ext ? nullptr : timing_begin(s);
    FV_HIP(fv::launch_finalize(c, partials, nullptr, single, 1, flags, Od, normpart, s));
    timing_end(t1, 1, s);
    return FV_OK;
  };
  if (ext) {
    rc = enqueue();
    if (rc) return rc;
    if (!(flags & FV_ASYNC)) FV_HIP(hipStreamSynchronize(s));
    return FV_OK;
  }
  const bool use_graph = graphs_enabled() && s != nullptr && (flags & FV_X_DEVICE) &&
                         (flags & FV_OUT_DEVICE) && !timing_enabled();
  GraphKey key;
  key.kind = 0;
  key.gmm = gmm->serial;
  key.precision = precision;
  key.flags = flags & kGraphFlags;
  key.path = (int)path + (gam_path ? 2 : 0);
  key.P = P;
  key.rows = N;
  key.n_items = n_items;
  key.n_groups = n_groups;
  key.X = Xd;
  key.out = Od;
  key.dev = ws->dev;
  key.pca = pca ? pca->serial : 0;
  key.cap = grid_cap(1 << 30) == (1 << 30) ? 0 : grid_cap(1 << 30);
  key.grid = gmm->batch_grid;
  key.variant = gmm->fused16_variant + 4 * fused16_env();
  rc = run_sequence(ws, key, use_graph, s, enqueue);
  if (rc) return rc;
  if (!(flags & FV_OUT_DEVICE))
    FV_HIP(hipMemcpyAsync(out, Od, out_len * 4, hipMemcpyDeviceToHost, s));
  if (!(flags & FV_ASYNC)) FV_HIP(hipStreamSynchronize(s));
  return FV_OK;
}

// fv_encode_batch, with the projection prologue when pca is non-null.
static int encode_batch_impl(const fv_gmm* gmm, const fv_pca* pca, const float* X,
                             const int64_t* offsets, int B, float* out, int precision,
                             unsigned flags, void* hip_stream) {
  if (!gmm || !offsets || B < 0 || (B > 0 && !out)) return FV_E_INVAL;
  if (const int fs = fv_form_status(gmm, precision)) return fs;
  if (flags & ~kAllFlags) return FV_E_INVAL;
  if (pca && (pca->D != gmm->D || pca->device != gmm->device)) return FV_E_INVAL;
  if (offsets[0] != 0) return FV_E_INVAL;
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] < offsets[b]) return FV_E_INVAL;
  if (B == 0) return FV_OK;
  const int64_t rows = offsets[B];
  if (rows > 0 && !X) return FV_E_INVAL;
  const fv::Consts c = call_consts(gmm, flags);
  const int Din = pca ? pca->Din : c.D;
  if (rows > ((int64_t)1 << 40) / std::max(Din, c.D)) return FV_E_UNSUPPORTED;

  // Frame-relative chunking: frame b's chunk j covers its rows [j*P, (j+1)*P).
  const Path path = choose_batch(gmm, precision);
  const int P = batch_chunk(gmm);
  std::vector<fv::Frame> frames((size_t)B);
  int64_t n_items64 = 0, n_groups64 = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = offsets[b + 1] - offsets[b];
    const int64_t ni = (n + P - 1) / P;
    const int64_t ng = (ni + fv::kGroupItems - 1) / fv::kGroupItems;
    frames[b] = fv::Frame{n, (int32_t)n_items64, (int32_t)ni, b, (int32_t)ng};
    n_items64 += ni;
    n_groups64 += ng;
  }
  if (n_items64 > (int64_t)1 << 30) return FV_E_UNSUPPORTED;
  const int n_items = (int)n_items64;
  const int n_groups = (int)n_groups64;

  DeviceGuard g(gmm->device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Workspace* ws = workspace_for(gmm->device, s);
  if (!ws) return FV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ws->mu);

  // The launch sequence is sized to the workspace's capacities (frames, items, chunk groups,
  // rows), which only grow (doubling), and the kernels read the batch's own sizes from the
  // Counts record at the head of the work table: one captured graph serves every batch that
  // fits the capacities, whatever its frame sizes.
  fv::BatchCaps& cp = ws->caps;
  cp.B = std::max(cp.B, grow_cap(cp.B, B, 8));
  cp.items = std::max(cp.items, grow_cap(cp.items, n_items, 64));
  cp.groups = std::max(cp.groups, grow_cap(cp.groups, n_groups, 8));
  cp.rows = std::max(cp.rows, grow_cap64(cp.rows, rows, (int64_t)1 << 16));
  const size_t out_len = (size_t)2 * c.K * c.D;
  const BatchLayout lay = batch_layout(c, path, cp, Din, flags, pca != nullptr);
  const size_t b_part = lay.part, b_norm = lay.norm, b_lse = lay.lse, b_cnt = lay.cnt;
  const size_t b_frames = lay.frames, b_items = lay.items;
  const size_t b_tab = lay.tab();
  const size_t b_x = lay.x, b_out = lay.out, b_y = lay.y;
  int rc = ensure_dev(ws, b_part + b_norm + b_lse + b_tab + b_x + b_out + b_y, s);
  if (rc) return rc;
  rc = ensure_pinned(ws, b_tab);
  if (rc) return rc;
  char* base = ws->dev;
  float* partials = reinterpret_cast<float*>(base);
  double* normpart = reinterpret_cast<double*>(base + b_part);
  float2* lse = reinterpret_cast<float2*>(base + b_part + b_norm);
  char* tab = base + b_part + b_norm + b_lse;
  const fv::Counts* dcounts = reinterpret_cast<const fv::Counts*>(tab);
  fv::Frame* dframes = reinterpret_cast<fv::Frame*>(tab + b_cnt);
  fv::Item* ditems = reinterpret_cast<fv::Item*>(tab + b_cnt + b_frames);
  const int32_t* dorder = reinterpret_cast<const int32_t*>(tab + b_cnt + b_frames + b_items);
  float* xdev = reinterpret_cast<float*>(tab + b_tab);
  float* odev = reinterpret_cast<float*>(tab + b_tab + b_x);
  float* ydev = reinterpret_cast<float*>(tab + b_tab + b_x + b_out);

  // work tables in pinned memory (same layout as on the device), then one H2D copy of the
  // whole capacity
  const int half = ws->pin_half;
  char* pin = ws->pinned + (size_t)half * ws->pin_cap;
  fv::Counts* hcounts = reinterpret_cast<fv::Counts*>(pin);
  fv::Frame* hframes = reinterpret_cast<fv::Frame*>(pin + b_cnt);
  fv::Item* hitems = reinterpret_cast<fv::Item*>(pin + b_cnt + b_frames);
  int32_t* horder = reinterpret_cast<int32_t*>(pin + b_cnt + b_frames + b_items);
  *hcounts = fv::Counts{rows, n_items, (int32_t)((rows + fv::kTile - 1) / fv::kTile), B, 0};
  // the finalize takes the frames with the most slots first (its longest workgroups start
  // first); each record keeps the frame's index in the batch
  for (int b = 0; b < B; ++b) hframes[b] = frames[b];
  std::stable_sort(hframes, hframes + B, [](const fv::Frame& a, const fv::Frame& b) {
    return a.nitems > b.nitems;
  });
  {
    int64_t i = 0;
    for (int b = 0; b < B; ++b) {
      for (int32_t q = 0; q < frames[b].nitems; ++q, ++i) {
        const int64_t r0 = (int64_t)q * P;
        const int64_t nr = std::min<int64_t>(P, frames[b].nrows - r0);
        hitems[i] = fv::Item{offsets[b] + r0, (int32_t)nr, 0};
      }
    }
    // the statistics launch takes the items largest first (full chunks, then every frame's
    // last, partial chunk by size), so the partial ones fill the end of the launch
    for (int32_t k = 0; k < n_items; ++k) horder[k] = k;
    std::stable_sort(horder, horder + n_items,
                     [&](int32_t a, int32_t b) { return hitems[a].nrows > hitems[b].nrows; });
  }
  const float* Xd = X;
  if (!(flags & FV_X_DEVICE) && rows > 0) {
    FV_HIP(hipMemcpyAsync(xdev, X, (size_t)rows * Din * 4, hipMemcpyHostToDevice, s));
    Xd = xdev;
  }
  if ((reinterpret_cast<uintptr_t>(Xd) & 3) != 0) return FV_E_INVAL;
  float* Od = (flags & FV_OUT_DEVICE) ? out : odev;
  const float* Fx = pca ? ydev : Xd;  // the encoder's input
  const bool vec_ok = (c.D % 4 == 0) && ((reinterpret_cast<uintptr_t>(Fx) & 15) == 0);
  fv::Consts cc = c;
  cc.cnt = dcounts;
  cc.queue = fv::ItemQueue{const_cast<int32_t*>(&dcounts->next), dorder};
  // The table copy, the projection (if any), one persistent statistics launch over the items
  // (grid = resident workgroups) or the two passes, then the finalize over the frame capacity
  // (slots past the batch exit at once).  Every grid depends on the capacities only.
  auto enqueue = [&]() -> int {
    FV_HIP(hipMemcpyAsync(tab, pin, b_tab, hipMemcpyHostToDevice, s));
    if (pca) {
      hipEvent_t tp = timing_begin(s);
      FV_HIP(fv::launch_project(pca->p, Xd, cp.rows, ydev, project_grid(gmm->device, cp.rows),
                                s, dcounts, precision != FV_PREC_FP32));
      timing_end(tp, 2, s);
    }
    hipEvent_t t0 = timing_begin(s);
    const int resident = gmm->batch_grid > 0 ? gmm->batch_grid : resident_fused(gmm->device, c.Wg);
    if (path == Path::kFused) {
      FV_HIP(run_stats(cc, precision, Fx, vec_ok, cp.rows, P, ditems, cp.items,
                       grid_cap(resident), partials, s));
    } else {
      // The two passes span component groups in blockIdx.y, which one counter cannot serve
      // (and the first pass walks tiles, not the table's items): static assignment.
      fv::Consts c2 = cc;
      c2.queue = fv::ItemQueue{nullptr, nullptr};
      const int tiles_cap = (int)((cp.rows + fv::kTile - 1) / fv::kTile);
      FV_HIP(run_lse(c2, precision, Fx, vec_ok, cp.rows, tiles_cap, grid_cap(resident), lse,
                     cp.rows, s));
      const int groups = normext_groups(c, precision);
      const int grid2 = grid_cap(xcd_grid((device_cu_count(gmm->device) + groups - 1) / groups));
      FV_HIP(run_normext(c2, precision, Fx, vec_ok, cp.rows, P, ditems, cp.items, grid2, lse,
                         cp.rows, partials, s));
    }
    timing_end(t0, 0, s);
    hipEvent_t t1 = timing_begin(s);
    FV_HIP(fv::launch_finalize(cc, partials, dframes, fv::Frame{0, 0, 0, 0, 0}, cp.B, flags, Od,
                               normpart, s));
    timing_end(t1, 1, s);
    return FV_OK;
  };
  // (a batch without rows runs directly: its X may be any pointer, even null, and there is
  // nothing to replay)
  const bool use_graph = graphs_enabled() && s != nullptr && (flags & FV_X_DEVICE) &&
                         (flags & FV_OUT_DEVICE) && !timing_enabled() && rows > 0;
  GraphKey key;
  key.kind = 1;
  key.gmm = gmm->serial;
  key.precision = precision;
  key.flags = flags & kGraphFlags;
  key.path = (int)path;
  key.P = P;
  key.rows = cp.rows;
  key.B = cp.B;
  key.n_items = cp.items;
  key.n_groups = cp.groups;
  key.X = Xd;
  key.out = Od;
  key.dev = ws->dev;
  key.pinned = pin;
  key.pca = pca ? pca->serial : 0;
  key.cap = grid_cap(1 << 30) == (1 << 30) ? 0 : grid_cap(1 << 30);
  key.grid = gmm->batch_grid;
  key.variant = gmm->fused16_variant + 4 * fused16_env();
  rc = run_sequence(ws, key, use_graph, s, enqueue);
  if (rc) return rc;
  FV_HIP(hipEventRecord(ws->pin_done[half], s));
  ws->pin_pending[half] = true;
  ws->pin_half = half ^ 1;
  if (!(flags & FV_OUT_DEVICE))
    FV_HIP(hipMemcpyAsync(out, Od, (size_t)B * out_len * 4, hipMemcpyDeviceToHost, s));
  if (!(flags & FV_ASYNC)) FV_HIP(hipStreamSynchronize(s));
  return FV_OK;
}

int fv_encode(const fv_gmm* gmm, const float* X, int64_t N, float* out, int precision,
              unsigned flags, void* hip_stream) {
  return encode_impl(gmm, nullptr, X, N, out, precision, flags, hip_stream);
}

}  // extern "C"

namespace fv {
int encode_on_scratch(const fv_gmm* gmm, const float* X, int64_t N, float* out, int precision,
                      unsigned flags, void* hip_stream, char* scratch, size_t scratch_bytes) {
  if (!gmm || !scratch) return FV_E_INVAL;
  if ((flags & (FV_X_DEVICE | FV_OUT_DEVICE)) != (FV_X_DEVICE | FV_OUT_DEVICE)) return FV_E_INVAL;
  return encode_impl(gmm, nullptr, X, N, out, precision, flags, hip_stream, scratch,
                     scratch_bytes);
}
}  // namespace fv

namespace fv {
int set_device(int device) {
  const hipError_t e = hipSetDevice(device);
  return e == hipSuccess ? FV_OK : hip_fail(e);
}

int device_error(hipError_t e) { return hip_fail(e); }
}  // namespace fv

extern "C" {

int fv_encode_batch(const fv_gmm* gmm, const float* X, const int64_t* offsets, int B, float* out,
                    int precision, unsigned flags, void* hip_stream) {
  return encode_batch_impl(gmm, nullptr, X, offsets, B, out, precision, flags, hip_stream);
}

int fv_encode_projected(const fv_gmm* gmm, const fv_pca* pca, const float* X, int64_t N,
                        float* out, int precision, unsigned flags, void* hip_stream) {
  if (!pca) return FV_E_INVAL;
  return encode_impl(gmm, pca, X, N, out, precision, flags, hip_stream);
}

int fv_encode_batch_projected(const fv_gmm* gmm, const fv_pca* pca, const float* X,
                              const int64_t* offsets, int B, float* out, int precision,
                              unsigned flags, void* hip_stream) {
  if (!pca) return FV_E_INVAL;
  return encode_batch_impl(gmm, pca, X, offsets, B, out, precision, flags, hip_stream);
}

int fv_encode_images(const fv_gmm* gmm, const fv_pca* pca, const float* images, int n_images,
                     int H, int W, int n_scales, const double* scales, int bin, int step,
                     float* out, int precision, unsigned flags, void* hip_stream) {
  if (!gmm || !pca || n_images < 0) return FV_E_INVAL;
  if (flags & ~kAllFlags) return FV_E_INVAL;
  if (pca->Din != fv::kDsiftDim || pca->D != gmm->D || pca->device != gmm->device)
    return FV_E_INVAL;
  if (const int fs = fv_form_status(gmm, precision)) return fs;
  const fv::DsiftPlan* p = nullptr;
  int rc = fv::dsift_plan(H, W, n_scales, scales, bin, step, &p);
  if (rc) return rc;
  if (n_images == 0) return FV_OK;
  if (!images || !out) return FV_E_INVAL;
  if ((size_t)n_images * (size_t)p->ndesc * fv::kDsiftDim * 4 > ((size_t)1 << 40))
    return FV_E_UNSUPPORTED;
  DeviceGuard g(gmm->device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  // descriptors of every image into the front end's workspace, then the projected batch
  // encode of the images' rows (one frame per image) on the same stream
  float* rows = nullptr;
  rc = fv::dsift_enqueue(*p, gmm->device, s, images, (flags & FV_X_DEVICE) != 0, n_images,
                         nullptr, &rows);
  if (rc) return rc;
  // A few images give the batched statistics launch too few chunks to fill the resident grid
  // (18 per 320 x 240 image): then each image is encoded on its own, with the single-frame
  // plan, which sizes its chunks to the GPU.
  const int64_t chunks = (p->ndesc + batch_chunk(gmm) - 1) / batch_chunk(gmm);
  if ((int64_t)n_images * chunks < resident_fused(gmm->device, gmm->c.Wg)) {
    const size_t out_len = (size_t)2 * gmm->K * gmm->D;
    for (int b = 0; b < n_images; ++b) {
      rc = encode_impl(gmm, pca, rows + (size_t)b * p->ndesc * fv::kDsiftDim, p->ndesc,
                       out + (size_t)b * out_len, precision, (flags | FV_X_DEVICE) | FV_ASYNC,
                       hip_stream);
      if (rc) return rc;
    }
    if (!(flags & FV_ASYNC)) FV_HIP(hipStreamSynchronize(s));
    return FV_OK;
  }
  std::vector<int64_t> offsets((size_t)n_images + 1);
  for (int b = 0; b <= n_images; ++b) offsets[(size_t)b] = (int64_t)b * p->ndesc;
  return encode_batch_impl(gmm, pca, rows, offsets.data(), n_images, out, precision,
                           flags | FV_X_DEVICE, hip_stream);
}

int fv_pca_load(int Din, int D, const float* A, const float* mean, int device, fv_pca** out) {
  if (!out) return FV_E_INVAL;
  *out = nullptr;
  if (Din < 1 || D < 1 || !A || !mean) return FV_E_INVAL;
  for (size_t i = 0; i < (size_t)D * Din; ++i)
    if (!finite_f(A[i])) return FV_E_INVAL;
  for (int i = 0; i < Din; ++i)
    if (!finite_f(mean[i])) return FV_E_INVAL;
  if (Din > fv::kMaxDin || D > fv::kMaxD) return FV_E_UNSUPPORTED;
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess) return hip_fail(de);
  if (device < 0 || device >= ndev) return FV_E_INVAL;

  fv::ProjConsts p{};
  p.Din = Din;
  p.D = D;
  p.S = (Din + 31) / 32 * 16;
  p.Dp = (D + 31) / 32 * 32;
  // operand rows k = 0..2S-1 (input features), columns c = 0..Dp-1 (outputs); bias = -A m in
  // double, rounded once
  std::vector<float> frag((size_t)2 * p.S * p.Dp, 0.f), bias((size_t)p.Dp, 0.f);
  for (int c = 0; c < D; ++c) {
    double am = 0.0;
    for (int k = 0; k < Din; ++k) {
      frag[(size_t)k * p.Dp + c] = A[(size_t)c * Din + k];
      am += (double)A[(size_t)c * Din + k] * (double)mean[k];
    }
    bias[c] = (float)(-am);
  }
  // the split form's bf16 hi/lo fragments: element e of (step s, half h, column c) is
  // A[c][16 s + 8 h + e]; hi = rne(a), lo = rne(a - hi) (a - hi exact in FP32)
  const int ns16 = (Din + 63) / 64 * 4;
  std::vector<uint16_t> fhi((size_t)ns16 * 2 * p.Dp * 8, 0), flo(fhi.size(), 0);
  for (int st = 0; st < ns16; ++st)
    for (int hh = 0; hh < 2; ++hh)
      for (int c = 0; c < D; ++c)
        for (int e = 0; e < 8; ++e) {
          const int k = 16 * st + 8 * hh + e;
          if (k >= Din) continue;
          const float a = A[(size_t)c * Din + k];
          const uint16_t hi = bf16_rne(a);
          const size_t o = (((size_t)st * 2 + hh) * p.Dp + c) * 8 + e;
          fhi[o] = hi;
          flo[o] = bf16_rne(a - bf16_to_f32(hi));
        }
  const size_t oF = 0, oB = align256(frag.size() * 4), oH = oB + align256(bias.size() * 4),
               oL = oH + align256(fhi.size() * 2), total = oL + align256(flo.size() * 2);
  DeviceGuard g(device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  std::unique_ptr<fv_pca> h(new (std::nothrow) fv_pca());
  if (!h) return FV_E_NOMEM;
  char* blk = nullptr;
  FV_HIP(hipMalloc(&blk, total));
  hipError_t e = hipMemcpy(blk + oF, frag.data(), frag.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(blk + oB, bias.data(), bias.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(blk + oH, fhi.data(), fhi.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(blk + oL, flo.data(), flo.size() * 2, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(blk);
    return hip_fail(e);
  }
  p.frag = reinterpret_cast<const float*>(blk + oF);
  p.bias = reinterpret_cast<const float*>(blk + oB);
  p.f16hi = reinterpret_cast<const uint16_t*>(blk + oH);
  p.f16lo = reinterpret_cast<const uint16_t*>(blk + oL);
  h->Din = Din;
  h->D = D;
  h->device = device;
  h->serial = g_next_serial.fetch_add(1);
  h->p = p;
  h->dev_block = blk;
  *out = h.release();
  return FV_OK;
}

int fv_pca_free(fv_pca* pca) {
  if (!pca) return FV_OK;
  int rc = FV_OK;
  {
    DeviceGuard g(pca->device);
    if (pca->dev_block) {
      hipError_t e = hipFree(pca->dev_block);
      if (e != hipSuccess) rc = hip_fail(e);
    }
  }
  delete pca;
  return rc;
}

int fv_pca_info(const fv_pca* pca, int* Din, int* D, int* device) {
  if (!pca) return FV_E_INVAL;
  if (Din) *Din = pca->Din;
  if (D) *D = pca->D;
  if (device) *device = pca->device;
  return FV_OK;
}

int fv_project(const fv_pca* pca, const float* X, int64_t N, float* Y, unsigned flags,
               void* hip_stream) {
  if (!pca || N < 0 || (N > 0 && (!X || !Y))) return FV_E_INVAL;
  if (flags & ~(FV_X_DEVICE | FV_OUT_DEVICE | FV_ASYNC | FV_PROJ_SPLIT16)) return FV_E_INVAL;
  if (N > ((int64_t)1 << 40) / std::max(pca->Din, pca->D)) return FV_E_UNSUPPORTED;
  if (N == 0) return FV_OK;
  DeviceGuard g(pca->device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Workspace* ws = workspace_for(pca->device, s);
  if (!ws) return FV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ws->mu);
  const size_t b_x = (flags & FV_X_DEVICE) ? 0 : align256((size_t)N * pca->Din * 4);
  const size_t b_y = (flags & FV_OUT_DEVICE) ? 0 : align256((size_t)N * pca->D * 4);
  int rc = ensure_dev(ws, b_x + b_y, s);
  if (rc) return rc;
  const float* Xd = X;
  if (!(flags & FV_X_DEVICE)) {
    float* xdev = reinterpret_cast<float*>(ws->dev);
    FV_HIP(hipMemcpyAsync(xdev, X, (size_t)N * pca->Din * 4, hipMemcpyHostToDevice, s));
    Xd = xdev;
  }
  if ((reinterpret_cast<uintptr_t>(Xd) & 3) != 0) return FV_E_INVAL;
  float* Yd = (flags & FV_OUT_DEVICE) ? Y : reinterpret_cast<float*>(ws->dev + b_x);
  if ((reinterpret_cast<uintptr_t>(Yd) & 3) != 0) return FV_E_INVAL;
  hipEvent_t tp = timing_begin(s);
  FV_HIP(fv::launch_project(pca->p, Xd, N, Yd, project_grid(pca->device, N), s, nullptr,
                            (flags & FV_PROJ_SPLIT16) != 0));
  timing_end(tp, 2, s);
  if (!(flags & FV_OUT_DEVICE))
    FV_HIP(hipMemcpyAsync(Y, Yd, (size_t)N * pca->D * 4, hipMemcpyDeviceToHost, s));
  if (!(flags & FV_ASYNC)) FV_HIP(hipStreamSynchronize(s));
  return FV_OK;
}

int fv_em_step(const fv_gmm* gmm, const float* X, int64_t N, int precision, float var_floor,
               unsigned flags, void* hip_stream, float* weights, float* means, float* variances,
               double* loglik) {
  if (!gmm || N < 1 || !X || !weights || !means || !variances || !loglik) return FV_E_INVAL;
  if (const int fs = fv_form_status(gmm, precision)) return fs;
  if (flags & ~(unsigned)FV_X_DEVICE) return FV_E_INVAL;
  if (!(var_floor >= 0.f) || !finite_f(var_floor)) return FV_E_INVAL;
  const fv::Consts c = call_consts(gmm, 0);
  if (N > ((int64_t)1 << 40) / c.D) return FV_E_UNSUPPORTED;
  DeviceGuard g(gmm->device);
  if (g.status() != hipSuccess) return hip_fail(g.status());
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Workspace* ws = workspace_for(gmm->device, s);
  if (!ws) return FV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ws->mu);

  // the encoder's two-pass path: the first pass gives the row normalisers (the likelihood),
  // the second the per-chunk sums S0, S1, S2
  const bool grouped = c.Kp > fv::kFusedMaxK;
  const int slices = c.Kp / fv::kCompsPerWave;
  const int P = grouped ? normext_single_chunk(N, gmm->device, normext_groups(c, precision))
                        : split_single_chunk(N, gmm->device, slices, sliced_round(c, precision));
  const int n_items = (int)((N + P - 1) / P);
  const int G = fv::lse_groups(c);
  const int nll = fv::em_loglik_blocks(N);
  const size_t KD = (size_t)c.K * c.D;
  const size_t b_part = align256((size_t)n_items * fv::slot_floats(c) * 4);
  const size_t b_lse = align256((size_t)G * N * 8);
  const size_t b_out = align256((c.K + 2 * KD) * 4);
  const size_t b_ll = align256((size_t)nll * 8);
  const size_t b_x = (flags & FV_X_DEVICE) ? 0 : align256((size_t)N * c.D * 4);
  int rc = ensure_dev(ws, b_part + b_lse + b_out + b_ll + b_x, s);
  if (rc) return rc;
  char* base = ws->dev;
  float* partials = reinterpret_cast<float*>(base);
  float2* lse = reinterpret_cast<float2*>(base + b_part);
  float* odev = reinterpret_cast<float*>(base + b_part + b_lse);
  double* lldev = reinterpret_cast<double*>(base + b_part + b_lse + b_out);
  float* xdev = reinterpret_cast<float*>(base + b_part + b_lse + b_out + b_ll);
  const float* Xd = X;
  if (!(flags & FV_X_DEVICE)) {
    FV_HIP(hipMemcpyAsync(xdev, X, (size_t)N * c.D * 4, hipMemcpyHostToDevice, s));
    Xd = xdev;
  }
  if ((reinterpret_cast<uintptr_t>(Xd) & 3) != 0) return FV_E_INVAL;
  const bool vec_ok = (c.D % 4 == 0) && ((reinterpret_cast<uintptr_t>(Xd) & 15) == 0);
  const int n_tiles = (int)((N + fv::kTile - 1) / fv::kTile);
  const int grid1 = grid_cap(std::min(n_tiles, resident_fused(gmm->device, c.Wg)));
  FV_HIP(run_lse(c, precision, Xd, vec_ok, N, n_tiles, grid1, lse, N, s));
  const int grid2 = grid_cap(xcd_grid(n_items));
  if (grouped)
    FV_HIP(run_normext(c, precision, Xd, vec_ok, N, P, nullptr, n_items, grid2, lse, N,
                       partials, s));
  else
    FV_HIP(run_sliced(c, precision, Xd, vec_ok, N, P, nullptr, n_items, grid2, lse, N,
                      partials, s));
  FV_HIP(fv::launch_em(c, partials, n_items, N, var_floor, lse, N, odev, odev + c.K,
                       odev + c.K + KD, lldev, s));
  std::vector<float> hout(c.K + 2 * KD);
  std::vector<double> hll((size_t)nll);
  FV_HIP(hipMemcpyAsync(hout.data(), odev, hout.size() * 4, hipMemcpyDeviceToHost, s));
  FV_HIP(hipMemcpyAsync(hll.data(), lldev, hll.size() * 8, hipMemcpyDeviceToHost, s));
  FV_HIP(hipStreamSynchronize(s));
  std::memcpy(weights, hout.data(), (size_t)c.K * 4);
  std::memcpy(means, hout.data() + c.K, KD * 4);
  std::memcpy(variances, hout.data() + c.K + KD, KD * 4);
  double ll2 = 0.0;
  for (double v : hll) ll2 += v;
  // logits are log2-scaled and leave out the -D/2 ln(2 pi) of every Gaussian density
  *loglik = ll2 * 0.69314718055994530942 - (double)N * 0.5 * c.D * 1.8378770664093454836;
  return FV_OK;
}

}  // extern "C"
