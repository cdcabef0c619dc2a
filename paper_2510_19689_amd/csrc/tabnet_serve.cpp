// Serving runtime: continuous batching of variable-row requests onto the fused forward.
//
// The paper serves TabNet per invocation with a batch size chosen at invocation time
// (Sec. III-B) and names dynamic batching as its next optimisation (Sec. VI-D).  Here:
//
//   submit (any thread)  ->  pending queue (FIFO)
//   scheduler thread     ->  admits pending requests in order while their bytes fit the
//                            budget; packs the admitted rows of the oldest request's model
//                            (a request may be split) into a free slot's pinned input
//                            buffer; the executor enqueues copy-in, the forward and
//                            copy-out on the slot's stream
//   completion thread    ->  takes slots in launch order, waits for their copy-out,
//                            copies each slice to its request's buffers, completes
//                            requests, returns bytes to the budget and the slot to the pool
//
// The device work sits behind an Executor interface: the HIP executor owns the streams,
// device and pinned buffers and (optionally) one captured graph per slot and model; a
// fake executor lets the scheduling logic run on a machine without a GPU.
#include "tabnet_serve.hpp"

#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace tabnet {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

namespace {

enum class ReqState { Pending, Admitted, Done, Cancelled, Failed };

struct Request {
  uint64_t id;
  int model;
  int64_t rows;
  std::unique_ptr<float[]> X;    // copied at submit
  float* logits;
  float* magg;
  float* msteps;                 // may be null
  int64_t arrival_ns;
  uint64_t bytes;
  int64_t rows_launched = 0;
  int64_t rows_done = 0;
  int segs_inflight = 0;         // segments launched whose completion has not been handled
  bool failing = false;          // a segment failed; Failed once no segment is in flight
  ReqState state = ReqState::Pending;
};

struct Segment {                 // rows [src_row, src_row + rows) of a request, at slot row dst_row
  std::shared_ptr<Request> req;
  int64_t src_row, rows, dst_row;
};

struct Launch {
  int slot;
  int model;
  int64_t rows;
  std::vector<Segment> segs;
};

// Copy with non-temporal stores: the destination's cache lines are written without being
// read first (an ordinary store fetches each line it writes), so a large scatter moves a
// third fewer bytes through memory and leaves the caches alone.  The destination's head
// up to 32-byte alignment and the tail go through memcpy; the fence orders the streaming
// stores before whatever the caller does next (signalling completion).
__attribute__((target("avx2"))) static void copy_stream_avx2(char* dst, const char* src, size_t n) {
  const size_t head = std::min(n, (size_t)((32 - (reinterpret_cast<uintptr_t>(dst) & 31)) & 31));
  std::memcpy(dst, src, head);
  dst += head;
  src += head;
  n -= head;
  size_t i = 0;
  for (; i + 128 <= n; i += 128) {
    const __m256i a = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(src + i));
    const __m256i b = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(src + i + 32));
    const __m256i c = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(src + i + 64));
    const __m256i d = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(src + i + 96));
    _mm256_stream_si256(reinterpret_cast<__m256i*>(dst + i), a);
    _mm256_stream_si256(reinterpret_cast<__m256i*>(dst + i + 32), b);
    _mm256_stream_si256(reinterpret_cast<__m256i*>(dst + i + 64), c);
    _mm256_stream_si256(reinterpret_cast<__m256i*>(dst + i + 96), d);
  }
  for (; i + 32 <= n; i += 32)
    _mm256_stream_si256(reinterpret_cast<__m256i*>(dst + i),
                        _mm256_loadu_si256(reinterpret_cast<const __m256i*>(src + i)));
  std::memcpy(dst + i, src + i, n - i);
  _mm_sfence();
}

static void copy_bytes(void* dst, const void* src, size_t n) {
  static const bool avx2 = __builtin_cpu_supports("avx2");
  if (avx2 && n >= 4096)
    copy_stream_avx2(static_cast<char*>(dst), static_cast<const char*>(src), n);
  else
    std::memcpy(dst, src, n);
}

// Host copies of the serving path.  A launch's gather (request rows into the pinned input
// buffer) and scatter (outputs into each request's buffers) are batches of copies; a batch
// is cut into pieces of at most kPiece bytes (64-byte aligned) and shared by the worker
// threads and the calling thread, which waits for all of them.  At ten thousand requests
// per second with step masks the scatter alone is tens of GB/s, more than one thread's
// memcpy.
class CopyPool {
 public:
  static constexpr size_t kPiece = 256 << 10;

  struct Item {
    void* dst;
    const void* src;
    size_t bytes;
  };

  explicit CopyPool(int workers) {
    for (int i = 0; i < workers; ++i) thr_.emplace_back([this] { run(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : thr_) t.join();
  }
  void copy(void* dst, const void* src, size_t bytes) { copy_many({Item{dst, src, bytes}}); }

  void copy_many(const std::vector<Item>& items) {
    size_t total = 0;
    for (const Item& it : items) total += it.bytes;
    if (thr_.empty() || total < kPiece) {
      for (const Item& it : items) copy_bytes(it.dst, it.src, it.bytes);
      return;
    }
    Latch latch;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (const Item& it : items)
        for (size_t off = 0; off < it.bytes; off += kPiece) {
          jobs_.push_back(Job{static_cast<char*>(it.dst) + off, static_cast<const char*>(it.src) + off,
                              std::min(kPiece, it.bytes - off), &latch});
          ++latch.n;
        }
    }
    cv_.notify_all();
    // the calling thread takes pieces too (any batch's: they are all short)
    for (;;) {
      Job j;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (jobs_.empty()) break;
        j = jobs_.front();
        jobs_.pop_front();
      }
      finish(j);
    }
    std::unique_lock<std::mutex> lk(latch.m);
    latch.cv.wait(lk, [&] { return latch.n == 0; });
  }

 private:
  struct Latch {
    std::mutex m;
    std::condition_variable cv;
    int n = 0;
  };
  struct Job {
    char* dst;
    const char* src;
    size_t bytes;
    Latch* latch;
  };
  static void finish(const Job& j) {
    copy_bytes(j.dst, j.src, j.bytes);
    // the waiter may destroy the latch as soon as it sees n == 0: touch it only here
    std::lock_guard<std::mutex> ll(j.latch->m);
    if (--j.latch->n == 0) j.latch->cv.notify_all();
  }
  void run() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || !jobs_.empty(); });
      if (jobs_.empty()) return;   // stopping, nothing left
      const Job j = jobs_.front();
      jobs_.pop_front();
      lk.unlock();
      finish(j);
      lk.lock();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Job> jobs_;
  bool stop_ = false;
  std::vector<std::thread> thr_;
};

}  // namespace

struct ServerImpl {
  std::vector<ModelInfo> models;
  Executor* exec = nullptr;
  tabnet_serve_opts opts;
  uint64_t budget;
  int64_t max_rows;
  int nslots;

  std::mutex mu;
  std::condition_variable cv_sched, cv_comp, cv_done;
  std::deque<std::shared_ptr<Request>> pending;      // not yet admitted
  std::deque<std::shared_ptr<Request>> admitted;     // admitted, rows left to launch
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
  std::deque<Launch> inflight;                       // launch order
  std::vector<int> free_slots;
  uint64_t next_id = 1;
  uint64_t inflight_bytes = 0, peak_bytes = 0;
  bool stopping = false, sched_exited = false;
  int waiters = 0;               // threads inside server_wait

  // statistics since the last reset
  uint64_t n_sub = 0, n_adm = 0, n_done = 0, n_rej = 0, n_cancel = 0, rows_done = 0, launches = 0;
  uint64_t launched_rows = 0;
  int64_t first_arrival = 0, last_done = 0;
  std::vector<double> lat_us;
  struct PerModel {              // the same statistics for one model's requests and launches
    uint64_t n_sub = 0, n_adm = 0, n_done = 0, n_rej = 0, rows_done = 0, launches = 0, launched_rows = 0;
    int64_t first_arrival = 0, last_done = 0;
    std::vector<double> lat_us;
  };
  std::vector<PerModel> per_model;
  // per model: statistics (mean[D], M2[D], n) of masks_agg of its last launches, oldest first
  std::vector<std::deque<std::vector<double>>> mask_windows;

  CopyPool copies{6};
  std::thread sched_thr, comp_thr;

  uint64_t req_bytes(int model, int64_t rows) const {
    return (uint64_t)rows * models[model].bytes_per_row;
  }

  void scheduler() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // admission: FIFO, stop at the first request that does not fit
      while (!pending.empty() && inflight_bytes + pending.front()->bytes <= budget) {
        auto r = pending.front();
        pending.pop_front();
        r->state = ReqState::Admitted;
        inflight_bytes += r->bytes;
        peak_bytes = std::max(peak_bytes, inflight_bytes);
        ++n_adm;
        ++per_model[r->model].n_adm;
        admitted.push_back(r);
      }
      if (stopping && admitted.empty()) break;
      if (admitted.empty() || free_slots.empty()) {
        cv_sched.wait(lk);
        continue;
      }
      // The launch serves the model of the oldest admitted request and takes, in arrival
      // order, the rows of every admitted request of that model until it is full, so that
      // a mixed stream still forms large per-model batches.
      Launch L;
      L.slot = free_slots.back();
      free_slots.pop_back();
      L.model = admitted.front()->model;
      L.rows = 0;
      for (auto it = admitted.begin(); it != admitted.end() && L.rows < max_rows;) {
        auto r = *it;
        if (r->model != L.model) {
          ++it;
          continue;
        }
        const int64_t take = std::min(r->rows - r->rows_launched, max_rows - L.rows);
        L.segs.push_back(Segment{r, r->rows_launched, take, L.rows});
        ++r->segs_inflight;
        r->rows_launched += take;
        L.rows += take;
        if (r->rows_launched == r->rows)
          it = admitted.erase(it);
        else
          ++it;
      }
      lk.unlock();
      // gather the rows into the slot's input buffer and enqueue the launch
      const int D = models[L.model].cfg.D;
      float* in = exec->input(L.slot);
      std::vector<CopyPool::Item> gather;
      for (const Segment& sg : L.segs)
        gather.push_back({in + sg.dst_row * D, sg.req->X.get() + sg.src_row * D, (size_t)sg.rows * D * sizeof(float)});
      copies.copy_many(gather);
      const bool ok = exec->launch(L.slot, L.model, L.rows);
      lk.lock();
      ++launches;
      launched_rows += L.rows;
      ++per_model[L.model].launches;
      per_model[L.model].launched_rows += L.rows;
      if (!ok) {
        for (Segment& sg : L.segs) {
          --sg.req->segs_inflight;
          fail_request(sg.req);
        }
        free_slots.push_back(L.slot);
        continue;
      }
      inflight.push_back(std::move(L));
      cv_comp.notify_one();
    }
    sched_exited = true;
    cv_comp.notify_all();
  }

  // A segment of r failed (mu held).  Its rows not yet launched are dropped, and the
  // request is reported Failed only once none of its segments is in flight, so that no
  // copy-out can write to the caller's buffers after wait or poll has returned.
  void fail_request(const std::shared_ptr<Request>& r) {
    if (r->state != ReqState::Admitted) return;
    if (!r->failing) {
      r->failing = true;
      for (auto it = admitted.begin(); it != admitted.end(); ++it)
        if (*it == r) {
          admitted.erase(it);
          break;
        }
    }
    if (r->segs_inflight > 0) return;
    inflight_bytes -= r->bytes;
    r->state = ReqState::Failed;
    r->X.reset();
    cv_done.notify_all();
  }

  void completer() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (inflight.empty()) {
        if (sched_exited) break;
        cv_comp.wait(lk);
        continue;
      }
      Launch L = std::move(inflight.front());
      inflight.pop_front();
      // rows of a request that has failed elsewhere are not copied out (its buffers stay
      // valid until it is reported: it still counts this segment as in flight)
      std::vector<char> skip(L.segs.size());
      for (size_t k = 0; k < L.segs.size(); ++k) skip[k] = L.segs[k].req->failing;
      lk.unlock();
      const bool ok = exec->wait(L.slot);
      const ModelInfo& mi = models[L.model];
      const int D = mi.cfg.D, n_out = mi.cfg.n_out, S = mi.cfg.n_steps;
      std::vector<double> mstats;
      if (ok && opts.mask_stats_window > 0) {
        const double* ms = exec->out_mask_stats(L.slot);
        if (ms) mstats.assign(ms, ms + 2 * (size_t)D + 1);
      }
      if (ok) {
        const float* lo = exec->out_logits(L.slot);
        const float* ag = exec->out_agg(L.slot);
        const float* ms = exec->out_steps(L.slot);
        std::vector<CopyPool::Item> scatter;
        for (size_t k = 0; k < L.segs.size(); ++k) {
          if (skip[k]) continue;
          const Segment& sg = L.segs[k];
          Request& r = *sg.req;
          scatter.push_back({r.logits + sg.src_row * n_out, lo + sg.dst_row * n_out, (size_t)sg.rows * n_out * 4});
          scatter.push_back({r.magg + sg.src_row * D, ag + sg.dst_row * D, (size_t)sg.rows * D * 4});
          if (r.msteps && ms)
            for (int s = 0; s < S; ++s)
              scatter.push_back({r.msteps + ((int64_t)s * r.rows + sg.src_row) * D,
                                 ms + ((int64_t)s * L.rows + sg.dst_row) * D, (size_t)sg.rows * D * 4});
        }
        copies.copy_many(scatter);
      }
      const int64_t t = now_ns();
      lk.lock();
      if (!mstats.empty()) {
        auto& w = mask_windows[L.model];
        w.push_back(std::move(mstats));
        while ((int)w.size() > opts.mask_stats_window) w.pop_front();
      }
      for (const Segment& sg : L.segs) {
        Request& r = *sg.req;
        --r.segs_inflight;
        if (!ok || r.failing) {
          fail_request(sg.req);
          continue;
        }
        r.rows_done += sg.rows;
        if (r.rows_done == r.rows && r.state == ReqState::Admitted) {
          r.state = ReqState::Done;
          inflight_bytes -= r.bytes;
          ++n_done;
          rows_done += (uint64_t)r.rows;
          lat_us.push_back((double)(t - r.arrival_ns) * 1e-3);
          last_done = std::max(last_done, t);
          PerModel& pm = per_model[r.model];
          ++pm.n_done;
          pm.rows_done += (uint64_t)r.rows;
          pm.lat_us.push_back((double)(t - r.arrival_ns) * 1e-3);
          pm.last_done = std::max(pm.last_done, t);
          r.X.reset();
        }
      }
      free_slots.push_back(L.slot);
      cv_done.notify_all();
      cv_sched.notify_one();
    }
  }
};

// ------------------------------------------------------------------------------------
tabnet_status server_create(std::vector<ModelInfo> models, Executor* exec, const tabnet_serve_opts& o,
                            ServerImpl** out) {
  ServerImpl* s = new ServerImpl();
  s->models = std::move(models);
  s->exec = exec;
  s->opts = o;
  s->budget = o.mem_budget_bytes;
  s->max_rows = o.max_rows_per_launch;
  s->nslots = o.slots;
  s->mask_windows.resize(s->models.size());
  s->per_model.resize(s->models.size());
  for (int i = s->nslots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->sched_thr = std::thread([s] { s->scheduler(); });
  s->comp_thr = std::thread([s] { s->completer(); });
  *out = s;
  return TABNET_OK;
}

tabnet_status server_submit(ServerImpl* s, int model, const float* X, int64_t rows, float* logits,
                            float* magg, float* msteps, int64_t arrival_ns, uint64_t* id) {
  if (!s || !X || !logits || !magg || !id || rows <= 0 || model < 0 || model >= (int)s->models.size()) {
    set_error("tabnet_serve_submit: invalid argument");
    return TABNET_E_INVALID;
  }
  const ModelInfo& mi = s->models[model];
  auto r = std::make_shared<Request>();
  r->model = model;
  r->rows = rows;
  r->logits = logits;
  r->magg = magg;
  r->msteps = s->opts.with_step_masks ? msteps : nullptr;
  r->arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
  r->bytes = s->req_bytes(model, rows);
  if (r->bytes > s->budget) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->n_rej;
    ++s->per_model[model].n_rej;
    set_error("tabnet_serve_submit: request larger than the memory budget");
    return TABNET_E_ADMISSION;
  }
  const size_t nx = (size_t)rows * mi.cfg.D;
  r->X.reset(new float[nx]);
  s->copies.copy(r->X.get(), X, nx * sizeof(float));
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) {
    set_error("tabnet_serve_submit: server stopped");
    return TABNET_E_STOPPED;
  }
  r->id = s->next_id++;
  *id = r->id;
  if (s->n_sub == 0 || r->arrival_ns < s->first_arrival) s->first_arrival = r->arrival_ns;
  ++s->n_sub;
  auto& pm = s->per_model[model];
  if (pm.n_sub == 0 || r->arrival_ns < pm.first_arrival) pm.first_arrival = r->arrival_ns;
  ++pm.n_sub;
  s->live[r->id] = r;
  s->pending.push_back(r);
  s->cv_sched.notify_one();
  return TABNET_OK;
}

static tabnet_status state_status(ReqState st) {
  switch (st) {
    case ReqState::Done: return TABNET_OK;
    case ReqState::Cancelled: return TABNET_E_STOPPED;
    case ReqState::Failed: return TABNET_E_HIP;
    default: return TABNET_E_TIMEOUT;
  }
}

tabnet_status server_wait(ServerImpl* s, uint64_t id, int64_t timeout_us) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) {
    set_error("tabnet_serve_wait: unknown request id");
    return TABNET_E_INVALID;
  }
  std::shared_ptr<Request> r = it->second;
  auto finished = [&] { return r->state != ReqState::Pending && r->state != ReqState::Admitted; };
  ++s->waiters;
  bool ok = true;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, finished);
  } else {
    ok = s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished);
  }
  --s->waiters;
  s->cv_done.notify_all();
  if (!ok) {
    set_error("tabnet_serve_wait: timed out");
    return TABNET_E_TIMEOUT;
  }
  s->live.erase(id);
  const tabnet_status st = state_status(r->state);
  if (st != TABNET_OK) set_error("tabnet_serve_wait: request cancelled or failed");
  return st;
}

tabnet_status server_poll(ServerImpl* s, uint64_t id, int* done) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) {
    set_error("tabnet_serve_poll: unknown request id");
    return TABNET_E_INVALID;
  }
  const ReqState st = it->second->state;
  if (st == ReqState::Pending || st == ReqState::Admitted) {
    *done = 0;
    return TABNET_OK;
  }
  *done = 1;
  s->live.erase(it);
  return state_status(st);
}

static double pct(std::vector<double>& v, double p) {
  if (v.empty()) return 0.0;
  const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
  std::nth_element(v.begin(), v.begin() + k, v.end());
  return v[k];
}

static void fill_latency(std::vector<double>& lat, tabnet_serve_stats* o) {
  if (lat.empty()) return;
  double sum = 0, mx = 0;
  for (double x : lat) {
    sum += x;
    mx = std::max(mx, x);
  }
  o->mean_us = sum / (double)lat.size();
  o->max_us = mx;
  o->p50_us = pct(lat, 0.50);
  o->p99_us = pct(lat, 0.99);
  o->p999_us = pct(lat, 0.999);
}

tabnet_status server_model_stats(ServerImpl* s, int model, tabnet_serve_stats* o) {
  if (model < 0 || model >= (int)s->models.size()) {
    set_error("tabnet_serve_get_model_stats: bad model index");
    return TABNET_E_INVALID;
  }
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const ServerImpl::PerModel& pm = s->per_model[model];
    std::memset(o, 0, sizeof *o);
    o->submitted = pm.n_sub;
    o->admitted = pm.n_adm;
    o->completed = pm.n_done;
    o->rejected = pm.n_rej;
    o->rows_completed = pm.rows_done;
    o->launches = pm.launches;
    o->mean_rows_per_launch = pm.launches ? (double)pm.launched_rows / (double)pm.launches : 0.0;
    o->inflight_bytes = s->inflight_bytes;
    o->peak_inflight_bytes = s->peak_bytes;
    const double span = (double)(pm.last_done - pm.first_arrival) * 1e-9;
    o->rows_per_s = (pm.n_done && span > 0) ? (double)pm.rows_done / span : 0.0;
    lat = pm.lat_us;
  }
  fill_latency(lat, o);
  return TABNET_OK;
}

tabnet_status server_stats(ServerImpl* s, tabnet_serve_stats* o) {
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(o, 0, sizeof *o);
    o->submitted = s->n_sub;
    o->admitted = s->n_adm;
    o->completed = s->n_done;
    o->rejected = s->n_rej;
    o->cancelled = s->n_cancel;
    o->rows_completed = s->rows_done;
    o->launches = s->launches;
    o->mean_rows_per_launch = s->launches ? (double)s->launched_rows / (double)s->launches : 0.0;
    o->inflight_bytes = s->inflight_bytes;
    o->peak_inflight_bytes = s->peak_bytes;
    const double span = (double)(s->last_done - s->first_arrival) * 1e-9;
    o->rows_per_s = (s->n_done && span > 0) ? (double)s->rows_done / span : 0.0;
    lat = s->lat_us;
  }
  fill_latency(lat, o);
  return TABNET_OK;
}

tabnet_status server_reset_stats(ServerImpl* s) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->n_sub = s->n_adm = s->n_done = s->n_rej = s->n_cancel = s->rows_done = s->launches = 0;
  s->launched_rows = 0;
  s->first_arrival = s->last_done = 0;
  s->lat_us.clear();
  for (auto& pm : s->per_model) pm = ServerImpl::PerModel();
  s->peak_bytes = s->inflight_bytes;
  for (auto& w : s->mask_windows) w.clear();
  return TABNET_OK;
}

// Merges the window's per-launch statistics, oldest first, with the pairwise update of
// Chan, Golub and LeVeque: n = n_a + n_b, d = mean_b - mean_a, mean = mean_a + d n_b / n,
// M2 = M2_a + M2_b + d^2 n_a n_b / n.
tabnet_status server_mask_stats(ServerImpl* s, int model, double* mean, double* var, int64_t* rows) {
  if (model < 0 || model >= (int)s->models.size() || !mean || !var) {
    set_error("tabnet_serve_mask_stats: bad model index or NULL output");
    return TABNET_E_INVALID;
  }
  if (s->opts.mask_stats_window <= 0) {
    set_error("tabnet_serve_mask_stats: the server was started with mask_stats_window = 0");
    return TABNET_E_INVALID;
  }
  const int D = s->models[model].cfg.D;
  std::vector<double> m(D, 0.0), q(D, 0.0);
  double n = 0.0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (const std::vector<double>& e : s->mask_windows[model]) {
      const double nb = e[2 * (size_t)D];
      if (nb <= 0.0) continue;
      const double nn = n + nb, f = nb / nn;
      for (int d = 0; d < D; ++d) {
        if (n == 0.0) {
          m[d] = e[d];
          q[d] = e[D + d];
        } else {
          const double dm = e[d] - m[d];
          m[d] += dm * f;
          q[d] += e[D + d] + dm * dm * n * f;
        }
      }
      n = nn;
    }
  }
  for (int d = 0; d < D; ++d) {
    mean[d] = n > 0.0 ? m[d] : 0.0;
    var[d] = n > 0.0 ? q[d] / n : 0.0;
  }
  if (rows) *rows = (int64_t)n;
  return TABNET_OK;
}

tabnet_status server_stop(ServerImpl* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    for (auto& r : s->pending) {
      r->state = ReqState::Cancelled;
      ++s->n_cancel;
    }
    s->pending.clear();
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
  }
  s->sched_thr.join();     // drains the admitted rows
  s->comp_thr.join();      // completes the launches in flight
  {
    // every request is now finished; let threads blocked in server_wait leave first
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_done.wait(lk, [s] { return s->waiters == 0; });
  }
  delete s->exec;
  delete s;
  return TABNET_OK;
}

// The serving path's host copy of n bytes (for the test library's hooks).
void serve_copy(void* dst, const void* src, size_t n) { copy_bytes(dst, src, n); }

}  // namespace tabnet
