// libfv serving loop: continuous batching of frames of different sizes with device-memory
// budget admission, several concurrent launches on the server's own HIP streams, per-request
// timestamps and latency percentiles.
//
// Request life cycle:  submit (host copy into pinned staging, FIFO queue)
//   -> admit (scheduler: queue head joins the batch being formed while the batch fits the
//      frame/row limits and the in-flight device footprint stays within the budget)
//   -> launch (one stream: H2D of every frame, fv_encode_batch, D2H of every result, event)
//   -> done (event observed complete; budget released) -> poll (result copied out, consumed).
// Admission is strictly in arrival order, so no request can starve.  Because the batched
// encoder chunks each frame relative to its own first row, a frame's result is bitwise the
// same whether it runs alone or together with any other frames.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fv.h"
#include "fv_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// Host staging blocks in power-of-two size classes, reused across requests (pinned memory for
// the HIP executor, plain memory for the fake one).
class HostPool {
 public:
  explicit HostPool(bool pinned) : pinned_(pinned) {}
  ~HostPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) release(p);
  }
  void* get(size_t bytes, size_t* cls_out) {
    *cls_out = 0;
    if (bytes > ((size_t)1 << 46)) return nullptr;  // beyond any frame the encoder accepts
    size_t cls = 1u << 16;
    while (cls < bytes) cls <<= 1;
    *cls_out = cls;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& v = free_[cls];
      if (!v.empty()) {
        void* p = v.back();
        v.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (pinned_) {
      if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    } else {
      p = std::malloc(cls);
    }
    return p;
  }
  void put(void* p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_[cls].push_back(p);
  }

 private:
  void release(void* p) {
    if (pinned_)
      (void)hipHostFree(p);
    else
      std::free(p);
  }
  bool pinned_;
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
};

// Helper threads for the submit-side copy of a host frame into its pinned staging block: a
// copy of at least 2 MiB is split into parts of at least 1 MiB, which the helpers and the
// submitting thread copy concurrently; submit returns once every part is done (so the caller
// may reuse its buffer at once, as before).  One memcpy thread moves about 28 GB/s here, far
// below what the host's memory and the H2D link sustain.
class CopyPool {
 public:
  explicit CopyPool(int n) {
    for (int i = 0; i < n; ++i) threads_.emplace_back([this] { run(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  void copy(void* dst, const void* src, size_t bytes) {
    constexpr size_t kMin = (size_t)1 << 20;
    const size_t helpers = threads_.size();
    size_t parts = std::min(helpers + 1, bytes / kMin);
    if (parts < 2) {
      std::memcpy(dst, src, bytes);
      return;
    }
    Done done;
    done.left = (int)parts - 1;
    const size_t per = (bytes / parts + 255) & ~(size_t)255;
    char* d = static_cast<char*>(dst);
    const char* sp = static_cast<const char*>(src);
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = 1; i < parts; ++i) {
        const size_t off = i * per;
        const size_t n = off >= bytes ? 0 : std::min(per, bytes - off);
        tasks_.push_back(Task{d + off, sp + off, n, &done});
      }
    }
    cv_.notify_all();
    std::memcpy(d, sp, std::min(per, bytes));
    std::unique_lock<std::mutex> lk(done.mu);
    done.cv.wait(lk, [&] { return done.left == 0; });
  }

 private:
  struct Done {
    std::mutex mu;
    std::condition_variable cv;
    int left = 0;
  };
  struct Task {
    char* dst;
    const char* src;
    size_t n;
    Done* done;
  };
  void run() {
    for (;;) {
      Task t;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !tasks_.empty(); });
        if (tasks_.empty()) return;  // stopping, nothing left
        t = tasks_.front();
        tasks_.pop_front();
      }
      if (t.n) std::memcpy(t.dst, t.src, t.n);
      // notify under the lock: the submitter's record lives on its stack and may go away as
      // soon as it can take the lock after the count reaches zero
      std::lock_guard<std::mutex> lk(t.done->mu);
      --t.done->left;
      t.done->cv.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Task> tasks_;
  bool stop_ = false;
  std::vector<std::thread> threads_;
};

struct Request {
  uint64_t ticket = 0;
  int64_t rows = 0;
  float* xin = nullptr;          // pinned staging copy of a host frame
  size_t xin_cls = 0;
  const float* xdev = nullptr;   // or the caller's device-resident frame (not owned)
  float* out = nullptr;
  size_t out_cls = 0;
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  int status = FV_PENDING;
  int batch_frames = 0;
};

struct Lane {  // one stream and its device buffers
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  float* dX = nullptr;
  size_t dX_cap = 0;  // floats
  float* dOut = nullptr;
  size_t dOut_cap = 0;
  fv::BatchCaps caps;  // of the encoder workspace on this lane's stream
  size_t ws_bytes = 0; // device bytes of that workspace
  // Device bytes this lane holds against the budget: its buffers and encoder workspace (HIP
  // executor; kept between launches), or the estimate of the batch in flight (fake executor).
  size_t held = 0;
  bool busy = false;
  std::vector<Request*> batch;
  // what the admitted batch needs (HIP executor): buffer sizes and workspace capacities
  size_t need_x = 0, need_o = 0;
  fv::BatchCaps need_caps;
  double fake_done_at = 0;
  int fake_status = FV_OK;
};

}  // namespace

struct fv_server {
  const fv_gmm* gmm = nullptr;
  fv_server_config cfg{};
  int K = 0, D = 0;
  size_t out_len = 0;
  Clock::time_point t0;
  std::unique_ptr<HostPool> pool;
  std::unique_ptr<CopyPool> copier;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> table;
  std::deque<uint64_t> finished;
  std::vector<Lane> lanes;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread sched;

  // counters
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, launches = 0, rows_done = 0;
  int64_t cancelled = 0;
  size_t admitted = 0, peak_admitted = 0;
  std::vector<double> lat_ms;
  double busy_s = 0, busy_since = -1;
  int64_t fake_batches = 0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
};

namespace {

// What lane L would hold after taking a batch of frames of these sizes: its buffers and its
// encoder workspace grown (never shrunk) to fit the batch (HIP executor), or the batch's
// device footprint estimate (fake executor, which holds nothing between batches).
struct Need {
  size_t bytes = 0, x = 0, o = 0;  // x, o in floats
  fv::BatchCaps caps;
};

Need lane_need(const fv_server* s, const Lane& L, const std::vector<int64_t>& sizes) {
  Need n;
  int64_t rows = 0;
  for (int64_t r : sizes) rows += r;
  if (s->cfg.executor == FV_EXEC_FAKE || !s->gmm) {
    for (int64_t r : sizes) n.bytes += (size_t)r * s->D * 4 + s->out_len * 4;
    return n;
  }
  n.x = std::max(L.dX_cap, (size_t)rows * s->D);
  n.o = std::max(L.dOut_cap, sizes.size() * s->out_len);
  n.caps = fv::caps_max(L.caps, fv::batch_need(s->gmm, sizes.data(), (int)sizes.size()));
  n.bytes = (n.x + n.o) * 4 + fv::batch_caps_bytes(s->gmm, s->cfg.precision, n.caps);
  return n;
}

size_t held_by_others(const fv_server* s, const Lane& L) {
  size_t n = 0;
  for (const Lane& M : s->lanes)
    if (&M != &L) n += M.held;
  return n;
}

void update_admitted(fv_server* s) {
  size_t n = 0;
  for (const Lane& L : s->lanes) n += L.held;
  s->admitted = n;
  s->peak_admitted = std::max(s->peak_admitted, n);
}

// Frees an idle lane's buffers and encoder workspace (HIP executor), so that its device memory
// no longer counts against the budget.
int release_lane(fv_server* s, Lane& L) {
  if (s->cfg.executor != FV_EXEC_HIP) {
    L.held = 0;
    return FV_OK;
  }
  int rc = fv_stream_release(s->gmm->device, L.stream);
  if (L.dX && hipFree(L.dX) != hipSuccess) rc = FV_E_DEVICE;
  if (L.dOut && hipFree(L.dOut) != hipSuccess) rc = FV_E_DEVICE;
  L.dX = L.dOut = nullptr;
  L.dX_cap = L.dOut_cap = 0;
  L.caps = fv::BatchCaps{};
  L.ws_bytes = 0;
  L.held = 0;
  return rc;
}

void finish_request(fv_server* s, Request* r, int status, double t) {
  r->status = status;
  r->t_done = t;
  if (status == FV_OK) {
    ++s->completed;
    s->rows_done += r->rows;
    if (s->lat_ms.size() < (1u << 22)) s->lat_ms.push_back((r->t_done - r->t_submit) * 1e-3);
  } else {
    ++s->failed;
  }
  s->finished.push_back(r->ticket);
}

// Launch one admitted batch on lane `L` (called without the server lock).
int launch(fv_server* s, Lane& L) {
  if (s->cfg.executor == FV_EXEC_FAKE) {
    int64_t rows = 0;
    for (Request* r : L.batch) rows += r->rows;
    ++s->fake_batches;
    L.fake_status = (s->cfg.fake_fail_every > 0 && s->fake_batches % s->cfg.fake_fail_every == 0)
                        ? FV_E_DEVICE
                        : FV_OK;
    for (Request* r : L.batch) std::memset(r->out, 0, s->out_len * 4);
    L.fake_done_at = s->now_us() + s->cfg.fake_us_per_krow * (double)rows / 1000.0;
    return FV_OK;
  }
  const int D = s->D;
  const int B = (int)L.batch.size();
  std::vector<int64_t> off((size_t)B + 1, 0);
  for (int b = 0; b < B; ++b) off[b + 1] = off[b] + L.batch[b]->rows;
  // grow the lane to exactly what admission counted for this batch
  if (L.need_x > L.dX_cap) {
    if (L.dX) {
      if (hipStreamSynchronize(L.stream) != hipSuccess || hipFree(L.dX) != hipSuccess) return FV_E_DEVICE;
      L.dX = nullptr;
      L.dX_cap = 0;
    }
    if (hipMalloc(&L.dX, L.need_x * 4) != hipSuccess) return FV_E_NOMEM;
    L.dX_cap = L.need_x;
  }
  if (L.need_o > L.dOut_cap) {
    if (L.dOut) {
      if (hipStreamSynchronize(L.stream) != hipSuccess || hipFree(L.dOut) != hipSuccess) return FV_E_DEVICE;
      L.dOut = nullptr;
      L.dOut_cap = 0;
    }
    if (hipMalloc(&L.dOut, L.need_o * 4) != hipSuccess) return FV_E_NOMEM;
    L.dOut_cap = L.need_o;
  }
  if (!(L.need_caps == L.caps) || L.ws_bytes == 0) {
    size_t wb = 0;
    const int rc = fv::batch_reserve(s->gmm, s->cfg.precision, L.stream, L.need_caps, &wb);
    if (rc != FV_OK) return rc;
    L.caps = L.need_caps;
    L.ws_bytes = wb;
  }
  for (int b = 0; b < B; ++b) {
    const Request* r = L.batch[b];
    if (r->rows > 0 &&
        hipMemcpyAsync(L.dX + (size_t)off[b] * D, r->xdev ? r->xdev : r->xin, (size_t)r->rows * D * 4,
                       r->xdev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, L.stream) != hipSuccess)
      return FV_E_DEVICE;
  }
  const unsigned fl = FV_X_DEVICE | FV_OUT_DEVICE | FV_ASYNC |
                      (s->cfg.flags & (FV_NO_POWER_NORM | FV_NO_L2_NORM | FV_THRESHOLD));
  int rc = fv_encode_batch(s->gmm, L.dX, off.data(), B, L.dOut, s->cfg.precision, fl, L.stream);
  if (rc != FV_OK) return rc;
  for (int b = 0; b < B; ++b)
    if (hipMemcpyAsync(L.batch[b]->out, L.dOut + (size_t)b * s->out_len, s->out_len * 4,
                       hipMemcpyDeviceToHost, L.stream) != hipSuccess)
      return FV_E_DEVICE;
  if (hipEventRecord(L.done, L.stream) != hipSuccess) return FV_E_DEVICE;
  return FV_OK;
}

// 0 = running, 1 = done ok, <0 = failed
int lane_state(fv_server* s, Lane& L) {
  if (s->cfg.executor == FV_EXEC_FAKE) {
    if (s->now_us() < L.fake_done_at) return 0;
    return L.fake_status == FV_OK ? 1 : L.fake_status;
  }
  const hipError_t e = hipEventQuery(L.done);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return FV_E_DEVICE;
}

void scheduler(fv_server* s) {
  if (s->cfg.executor == FV_EXEC_HIP) (void)hipSetDevice(s->gmm->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const double t = s->now_us();
    // 1. completions
    bool any_busy = false;
    for (Lane& L : s->lanes) {
      if (!L.busy) continue;
      const int st = lane_state(s, L);
      if (st == 0) {
        any_busy = true;
        continue;
      }
      for (Request* r : L.batch) finish_request(s, r, st == 1 ? FV_OK : st, t);
      if (s->cfg.executor != FV_EXEC_HIP) {  // the fake executor holds nothing between batches
        L.held = 0;
        update_admitted(s);
      }
      L.batch.clear();
      L.busy = false;
      s->cv_done.notify_all();
    }
    if (!any_busy && s->busy_since >= 0) {
      s->busy_s += (t - s->busy_since) * 1e-6;
      s->busy_since = -1;
    }
    // 2. deadlines of requests still waiting for admission
    if (s->cfg.deadline_ms > 0) {
      while (!s->queue.empty() && t - s->queue.front()->t_submit > s->cfg.deadline_ms * 1e3) {
        Request* r = s->queue.front();
        s->queue.pop_front();
        finish_request(s, r, FV_E_TIMEOUT, t);
        s->cv_done.notify_all();
      }
    }
    if (s->stop && s->queue.empty() && !any_busy) break;
    // 3. admission: FIFO into free lanes while frames, rows and budget allow.  With a batching
    //    window, a launch that could not be filled yet waits for its oldest request to age.
    bool launched = false;
    double window_left_us = 0;
    if (s->cfg.batch_window_us > 0 && !s->queue.empty() && !s->stop) {
      int64_t qrows = 0;
      for (const Request* r : s->queue) qrows += r->rows;
      const double age = t - s->queue.front()->t_submit;
      if ((int)s->queue.size() < s->cfg.max_batch_frames && qrows < s->cfg.max_batch_rows &&
          age < s->cfg.batch_window_us)
        window_left_us = s->cfg.batch_window_us - age;
    }
    // idle lanes, those holding the most device memory first (their buffers are reused)
    std::vector<Lane*> order;
    for (Lane& L : s->lanes)
      if (!L.busy) order.push_back(&L);
    std::stable_sort(order.begin(), order.end(),
                     [](const Lane* a, const Lane* b) { return a->held > b->held; });
    const size_t budget = s->cfg.hbm_budget_bytes;
    for (Lane* Lp : order) {
      Lane& L = *Lp;
      if (window_left_us > 0 || s->queue.empty()) break;
      std::vector<int64_t> sizes;
      int64_t rows = 0;
      Need need;
      for (int attempt = 0; attempt < 2 && L.batch.empty(); ++attempt) {
        sizes.clear();
        rows = 0;
        while (!s->queue.empty() && (int)sizes.size() < s->cfg.max_batch_frames) {
          Request* r = s->queue.front();
          if (!sizes.empty() && rows + r->rows > s->cfg.max_batch_rows) break;
          sizes.push_back(r->rows);
          const Need n = lane_need(s, L, sizes);
          if (budget > 0 && held_by_others(s, L) + n.bytes > budget) {
            sizes.pop_back();
            break;
          }
          need = n;
          rows += r->rows;
          s->queue.pop_front();
          r->t_admit = t;
          L.batch.push_back(r);
        }
        if (!L.batch.empty() || attempt > 0) break;
        // The head does not fit beside what the lanes hold: free the other idle lanes' memory,
        // or this lane's own when nothing else is held and nothing runs; then try once more.
        std::vector<Lane*> victims;
        bool running = false;
        for (Lane& M : s->lanes) {
          running |= M.busy;
          if (&M != &L && !M.busy && M.held > 0) victims.push_back(&M);
        }
        if (victims.empty() && !running && L.held > 0) victims.push_back(&L);
        if (victims.empty()) break;
        for (Lane* M : victims) M->busy = true;  // nothing else takes them meanwhile
        lk.unlock();
        for (Lane* M : victims) (void)release_lane(s, *M);
        lk.lock();
        for (Lane* M : victims) M->busy = false;
        update_admitted(s);
      }
      if (L.batch.empty()) {
        bool running = false;
        for (Lane& M : s->lanes) running |= M.busy;
        if (!running && !s->queue.empty() && budget > 0) {
          // nothing holds memory and nothing runs, yet the head does not fit: it never will
          Request* r = s->queue.front();
          s->queue.pop_front();
          ++s->rejected;
          finish_request(s, r, FV_E_BUDGET, t);
          s->cv_done.notify_all();
          launched = true;
        }
        break;  // keep arrival order
      }
      L.busy = true;
      L.held = need.bytes;
      L.need_x = need.x;
      L.need_o = need.o;
      L.need_caps = need.caps;
      update_admitted(s);
      ++s->launches;
      for (Request* r : L.batch) r->batch_frames = (int)L.batch.size();
      if (s->busy_since < 0) s->busy_since = t;
      lk.unlock();
      const int rc = launch(s, L);
      const double ts = s->now_us();
      lk.lock();
      if (s->cfg.executor == FV_EXEC_HIP) {
        L.held = (L.dX_cap + L.dOut_cap) * 4 + L.ws_bytes;  // what the lane really holds
        update_admitted(s);
      }
      for (Request* r : L.batch) r->t_start = ts;
      if (rc != FV_OK) {  // this batch fails; other requests continue
        if (s->cfg.executor == FV_EXEC_HIP) {
          lk.unlock();
          (void)hipStreamSynchronize(L.stream);  // no copy may still touch the staging blocks
          lk.lock();
        } else {
          L.held = 0;
          update_admitted(s);
        }
        for (Request* r : L.batch) finish_request(s, r, rc, ts);
        L.batch.clear();
        L.busy = false;
        s->cv_done.notify_all();
      }
      launched = true;
    }
    if (launched) continue;
    // 4. wait for work or for a running launch to finish
    bool busy_now = false;
    for (Lane& L : s->lanes) busy_now |= L.busy;
    if (window_left_us > 0)
      s->cv_work.wait_for(lk, std::chrono::duration<double, std::micro>(
                                  busy_now ? std::min(window_left_us, 20.0) : window_left_us));
    else if (busy_now)
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else if (s->queue.empty() && !s->stop)
      s->cv_work.wait(lk);
    else if (!s->queue.empty())
      s->cv_work.wait_for(lk, std::chrono::microseconds(200));
  }
}

void free_request(fv_server* s, Request* r) {
  s->pool->put(r->xin, r->xin_cls);
  s->pool->put(r->out, r->out_cls);
  delete r;
}

}  // namespace

extern "C" {

void fv_server_config_default(fv_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->precision = FV_PREC_FP32;
  c->max_queue = 4096;
  c->n_streams = 2;
  c->max_batch_frames = 64;
  c->max_batch_rows = 262144;
  c->executor = FV_EXEC_HIP;
  c->copy_threads = 3;
}

int fv_server_create(const fv_gmm* gmm, const fv_server_config* cfg, fv_server** out) {
  if (!out || !cfg) return FV_E_INVAL;
  *out = nullptr;
  fv_server_config c = *cfg;
  if (c.executor != FV_EXEC_HIP && c.executor != FV_EXEC_FAKE) return FV_E_INVAL;
  if (const int fs = fv_form_status(gmm, c.precision)) return fs;
  if (c.flags & ~(FV_NO_POWER_NORM | FV_NO_L2_NORM | FV_THRESHOLD)) return FV_E_INVAL;
  if (c.executor == FV_EXEC_HIP && !gmm) return FV_E_INVAL;
  if (!gmm && (c.fake_K < 1 || c.fake_D < 1)) return FV_E_INVAL;
  if (c.max_queue <= 0) c.max_queue = 4096;
  if (c.n_streams <= 0) c.n_streams = 2;
  if (c.n_streams > 16) c.n_streams = 16;
  if (c.max_batch_frames <= 0) c.max_batch_frames = 64;
  if (c.max_batch_rows <= 0) c.max_batch_rows = 262144;
  if (c.copy_threads < 0) c.copy_threads = 0;
  if (c.copy_threads > 16) c.copy_threads = 16;
  std::unique_ptr<fv_server> s(new (std::nothrow) fv_server());
  if (!s) return FV_E_NOMEM;
  s->gmm = gmm;
  s->cfg = c;
  s->K = gmm ? gmm->K : c.fake_K;
  s->D = gmm ? gmm->D : c.fake_D;
  s->out_len = (size_t)2 * s->K * s->D;
  s->t0 = Clock::now();
  s->pool.reset(new HostPool(c.executor == FV_EXEC_HIP));
  s->copier.reset(new (std::nothrow) CopyPool(c.copy_threads));
  if (!s->copier) return FV_E_NOMEM;
  s->lanes.resize((size_t)c.n_streams);
  if (c.executor == FV_EXEC_HIP) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(gmm->device) != hipSuccess) return FV_E_DEVICE;
    for (Lane& L : s->lanes) {
      if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
        for (Lane& M : s->lanes) {  // undo what was created
          if (M.done) (void)hipEventDestroy(M.done);
          if (M.stream) (void)hipStreamDestroy(M.stream);
        }
        (void)hipSetDevice(prev);
        return FV_E_DEVICE;
      }
    }
    (void)hipSetDevice(prev);
  }
  fv_server* raw = s.get();
  raw->sched = std::thread(scheduler, raw);
  *out = s.release();
  return FV_OK;
}

int fv_server_destroy(fv_server* s) {
  if (!s) return FV_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests not yet admitted are dropped
    while (!s->queue.empty()) {
      Request* r = s->queue.front();
      s->queue.pop_front();
      s->table.erase(r->ticket);
      free_request(s, r);
    }
  }
  s->cv_work.notify_all();
  if (s->sched.joinable()) s->sched.join();  // waits for in-flight launches
  for (auto& kv : s->table) free_request(s, kv.second);
  s->table.clear();
  int rc = FV_OK;
  if (s->cfg.executor == FV_EXEC_HIP) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->gmm->device);
    for (Lane& L : s->lanes) {
      // the encoder's cached buffers and graphs for this lane's stream
      if (L.stream && fv_stream_release(s->gmm->device, L.stream) != FV_OK) rc = FV_E_DEVICE;
      if (L.dX && hipFree(L.dX) != hipSuccess) rc = FV_E_DEVICE;
      if (L.dOut && hipFree(L.dOut) != hipSuccess) rc = FV_E_DEVICE;
      if (L.done) (void)hipEventDestroy(L.done);
      if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    (void)hipSetDevice(prev);
  }
  delete s;
  return rc;
}

namespace {

int submit_impl(fv_server* s, const float* X, int64_t N, uint64_t* ticket, bool device) {
  if (!s || !ticket || N < 0 || (N > 0 && !X)) return FV_E_INVAL;
  if (N > ((int64_t)1 << 40) / s->D) return FV_E_UNSUPPORTED;  // the encoder's row limit
  const std::vector<int64_t> one{N};
  if (s->cfg.hbm_budget_bytes > 0 && lane_need(s, Lane{}, one).bytes > s->cfg.hbm_budget_bytes) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rejected;
    return FV_E_BUDGET;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int)s->queue.size() >= s->cfg.max_queue) {
      ++s->rejected;
      return FV_E_AGAIN;
    }
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return FV_E_NOMEM;
  r->rows = N;
  if (N > 0 && device) {
    r->xdev = X;
  } else if (N > 0) {
    r->xin = static_cast<float*>(s->pool->get((size_t)N * s->D * 4, &r->xin_cls));
    if (!r->xin) return FV_E_NOMEM;
    s->copier->copy(r->xin, X, (size_t)N * s->D * 4);
  }
  r->out = static_cast<float*>(s->pool->get(s->out_len * 4, &r->out_cls));
  if (!r->out) {
    s->pool->put(r->xin, r->xin_cls);
    return FV_E_NOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now_us();
    *ticket = r->ticket;
    s->table[r->ticket] = r.get();
    s->queue.push_back(r.release());
    ++s->submitted;
  }
  s->cv_work.notify_one();
  return FV_OK;
}

}  // namespace

int fv_server_submit(fv_server* s, const float* X, int64_t N, uint64_t* ticket) {
  return submit_impl(s, X, N, ticket, false);
}

int fv_server_submit_device(fv_server* s, const float* X, int64_t N, uint64_t* ticket) {
  return submit_impl(s, X, N, ticket, true);
}

int fv_server_poll(fv_server* s, uint64_t ticket, float* out, fv_req_stats* st) {
  if (!s) return FV_E_INVAL;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return FV_E_NOTFOUND;
    r = it->second;
    if (r->status == FV_PENDING) return FV_PENDING;
    s->table.erase(it);
  }
  if (out && r->status == FV_OK) std::memcpy(out, r->out, s->out_len * 4);
  if (st) {
    st->t_submit_us = r->t_submit;
    st->t_admit_us = r->t_admit;
    st->t_start_us = r->t_start;
    st->t_done_us = r->t_done;
    st->rows = r->rows;
    st->batch_frames = r->batch_frames;
    st->status = r->status;
  }
  const int rc = r->status;
  free_request(s, r);
  return rc;
}

int fv_server_cancel(fv_server* s, uint64_t ticket) {
  if (!s) return FV_E_INVAL;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return FV_E_NOTFOUND;
    r = it->second;
    if (r->status == FV_PENDING) {
      // still waiting for admission?  (admitted requests have left the queue)
      auto q = std::find(s->queue.begin(), s->queue.end(), r);
      if (q == s->queue.end()) return FV_PENDING;
      s->queue.erase(q);
    } else {
      // finished, not polled: drop its completion notice
      auto f = std::find(s->finished.begin(), s->finished.end(), ticket);
      if (f != s->finished.end()) s->finished.erase(f);
    }
    s->table.erase(it);
    ++s->cancelled;
  }
  free_request(s, r);
  return FV_OK;
}

int fv_server_next_done(fv_server* s, double timeout_ms, uint64_t* ticket) {
  if (!s || !ticket) return FV_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return !s->finished.empty(); };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
    return FV_PENDING;
  *ticket = s->finished.front();
  s->finished.pop_front();
  return FV_OK;
}

int fv_server_get_stats(fv_server* s, fv_server_stats* st, int reset) {
  if (!s || !st) return FV_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->rejected = s->rejected;
  st->launches = s->launches;
  st->rows_done = s->rows_done;
  st->queued = (int)s->queue.size();
  int inflight = 0;
  for (const Lane& L : s->lanes) inflight += (int)L.batch.size();
  st->in_flight = inflight;
  st->admitted_bytes = s->admitted;
  st->peak_admitted_bytes = s->peak_admitted;
  std::vector<double> v = s->lat_ms;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::floor(p * (v.size() - 1) + 0.5));
    return v[i];
  };
  st->p50_ms = pct(0.50);
  st->p99_ms = pct(0.99);
  st->max_ms = v.empty() ? 0.0 : v.back();
  double busy = s->busy_s;
  if (s->busy_since >= 0) busy += (s->now_us() - s->busy_since) * 1e-6;
  st->busy_s = busy;
  st->cancelled = s->cancelled;
  st->graph_captures = 0;
  st->graph_replays = 0;
  if (s->cfg.executor == FV_EXEC_HIP) {
    for (const Lane& L : s->lanes) {
      int64_t c = 0, r = 0;
      fv::stream_graph_counts(s->gmm->device, L.stream, &c, &r);
      st->graph_captures += c;
      st->graph_replays += r;
    }
  }
  if (reset) {
    s->submitted = s->completed = s->failed = s->rejected = s->launches = s->rows_done = 0;
    s->cancelled = 0;
    s->lat_ms.clear();
    s->peak_admitted = s->admitted;
    s->busy_s = 0;
    if (s->busy_since >= 0) s->busy_since = s->now_us();
  }
  return FV_OK;
}

}  // extern "C"
