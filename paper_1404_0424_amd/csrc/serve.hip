// Native serving runtime (include/mimo_serve.h): request queue, HBM-budget
// admission, batched launches of same-class frames on HIP streams, and
// completion tracking, all in one scheduler thread per server.  Device work
// goes through the public entry points of mimo_cg.h, so a frame's outputs
// are bitwise those of a single call.  Host code only (no kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mimo_serve.h"
#include "launch.hpp"

namespace {

// ------------------------------------------------------------ DLPack ABI
// The exchange structs of the DLPack standard (v0.x layout), declared here
// so that outputs can be handed to frameworks without a copy.
struct DLDevice { int32_t device_type; int32_t device_id; };
struct DLDataType { uint8_t code; uint8_t bits; uint16_t lanes; };
struct DLTensor {
  void* data;
  DLDevice device;
  int32_t ndim;
  DLDataType dtype;
  int64_t* shape;
  int64_t* strides;
  uint64_t byte_offset;
};
struct DLManagedTensor {
  DLTensor dl_tensor;
  void* manager_ctx;
  void (*deleter)(DLManagedTensor*);
};
constexpr int32_t kDLROCM = 10;
constexpr uint8_t kDLFloat = 2, kDLComplex = 5;

// Errors go to the calling thread's mimo_last_error() message.
int fail(int status, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof(msg), fmt, ap);
  va_end(ap);
  mimo::set_last_error(msg);
  return status;
}

constexpr size_t kAlign = 256;
size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation; offsets, not pointers.
class Pool {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes ? bytes : 1);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    size_t start = off, len = bytes;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }
  size_t used() const { return used_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Channel {
  const void* H;
  int dtype;
  int64_t n_sc;
  int B, U;
  int64_t bytes;                // H and G, counted against the budget
  const void* G;                // caller's G = H^H H, or NULL
};

// Frames that read the channel's cached Gram: batched ones (approximate SINR
// uplink, every downlink) of channels with more than 8 users, where the
// cached form is bitwise the direct one (at U <= 8 the direct kernels form a
// packed Gram instead).
const void* frame_gram(const Channel& ch) { return ch.U > 8 ? ch.G : nullptr; }

struct Req {
  int64_t id = 0;
  int kind = 0;                 // 0 uplink, 1 downlink
  mimo_uplink_req up{};
  mimo_downlink_req dn{};
  Channel ch{};
  hipEvent_t ready = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  size_t out_bytes = 0, out2_bytes = 0, scratch_bytes = 0;
  size_t out_off = 0, scratch_off = 0;
  bool has_scratch = false;
  uint64_t key = 0;             // batch class; 0 = never batched
  int status = MIMO_OK;
  int holders = 0;              // caller's hold + DLPack tensors alive
  int S() const { return kind == 0 ? up.S : dn.S; }
  size_t need() const {
    return round_up(out_bytes + out2_bytes) + (has_scratch ? round_up(scratch_bytes) : 0);
  }
};

struct Launch {
  std::vector<Req*> reqs;
  int slot = 0;
  hipEvent_t done = nullptr;
  int status = MIMO_OK;
};

struct DoneRec {
  int64_t id;
  double t_submit, t_done;
  int64_t solves, llr_bits;
};

}  // namespace

struct mimo_server {
  // configuration
  mimo_server_config cfg{};
  int device = 0;
  // device resources
  char* pool_base = nullptr;
  hipStream_t streams[MIMO_SERVE_MAX_SLOTS] = {};
  hipEvent_t ref_event = nullptr;
  double t_ref = 0;             // host time of ref_event
  std::chrono::steady_clock::time_point origin;
  // state under mu
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new work or state change
  std::condition_variable cv_done;   // pollers / drain: completions
  Pool pool;
  std::unordered_map<int64_t, Channel> channels;
  int64_t channel_bytes = 0;
  std::deque<Req*> queue;
  std::vector<Launch*> inflight;
  std::vector<int> free_slots;
  std::deque<Req*> completed;        // not yet returned by poll
  std::unordered_map<int64_t, Req*> held;   // completed, outputs in the pool
  std::vector<DoneRec> records;
  std::vector<hipEvent_t> spare_events;
  int64_t next_id = 1;
  bool running = true, paused = false;
  double t_resume = -1;
  const Req* blocked = nullptr;
  int64_t budget_waits = 0, launches = 0, launched_frames = 0, peak_bytes = 0;
  std::thread thread;
  // DLPack deleters may run after destruction: they share this flag
  std::shared_ptr<std::atomic<bool>> alive = std::make_shared<std::atomic<bool>>(true);

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
  }
  void* ptr(size_t off) const { return pool_base + off; }
  void loop();
  bool admit_locked(std::vector<Launch*>& out);
  void run_launch(Launch* L);
  void finish_locked(Launch* L, double t_done);
  void free_request_locked(Req* r);
  hipEvent_t event_locked(unsigned flags);
};

namespace {

uint64_t batch_key(const Req& r) {
  if (r.kind == 0 && r.up.sinr_mode != MIMO_SINR_APPROX) return 0;
  uint64_t k = 1;
  k = k * 2 + (uint64_t)r.kind;
  k = k * 2 + (uint64_t)(r.ch.U <= 16);
  k = k * 4 + (uint64_t)r.ch.dtype;
  k = k * 16 + (uint64_t)(r.kind == 0 ? r.up.qam_bits : 0);
  k = k * 2 + (uint64_t)(r.kind == 0 ? r.up.scalar_prec : r.dn.scalar_prec);
  k = k * 2 + (uint64_t)(r.kind == 0 ? r.up.want_xhat : 0);
  return k;
}

}  // namespace

hipEvent_t mimo_server::event_locked(unsigned flags) {
  (void)flags;
  if (!spare_events.empty()) {
    hipEvent_t e = spare_events.back();
    spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void mimo_server::free_request_locked(Req* r) {
  pool.release(r->out_off, r->out_bytes + r->out2_bytes);
  delete r;
}

// Form launches from the queue head (called with mu held).  Returns true if
// anything was admitted.
bool mimo_server::admit_locked(std::vector<Launch*>& out) {
  bool any = false;
  while (!queue.empty() && !free_slots.empty() && !paused) {
    Req* head = queue.front();
    const int64_t cap = cfg.hbm_budget - channel_bytes;
    if ((int64_t)(pool.used() + head->need()) > cap) {
      if (blocked != head) {
        blocked = head;
        ++budget_waits;
      }
      break;
    }
    std::vector<Req*> group{head};
    size_t total = head->need();
    if (head->key != 0) {
      const size_t n = std::min<size_t>(queue.size(), (size_t)cfg.lookahead);
      for (size_t i = 1; i < n && (int)group.size() < cfg.max_batch; ++i) {
        Req* p = queue[i];
        if (p->key == head->key && (int64_t)(pool.used() + total + p->need()) <= cap) {
          group.push_back(p);
          total += p->need();
        }
      }
    }
    // pool offsets (first fit; fragmentation can refuse what the byte count
    // admits: then the head waits like any budget wait, and later members
    // that do not get memory stay queued)
    std::vector<Req*> got;
    for (Req* r : group) {
      if (!pool.alloc(r->out_bytes + r->out2_bytes, &r->out_off)) break;
      if (r->has_scratch && !pool.alloc(r->scratch_bytes, &r->scratch_off)) {
        pool.release(r->out_off, r->out_bytes + r->out2_bytes);
        break;
      }
      got.push_back(r);
    }
    if (got.empty()) {
      if (blocked != head) {
        blocked = head;
        ++budget_waits;
      }
      break;
    }
    group.swap(got);
    for (Req* r : group) {
      auto it = std::find(queue.begin(), queue.end(), r);
      if (it != queue.end()) queue.erase(it);
    }
    blocked = nullptr;
    const int64_t held_now = (int64_t)pool.used() + channel_bytes;
    if (held_now > peak_bytes) peak_bytes = held_now;
    Launch* L = new Launch;
    L->reqs = std::move(group);
    L->slot = free_slots.back();
    free_slots.pop_back();
    L->done = event_locked(0);
    const double t = now();
    for (Req* r : L->reqs) r->t_admit = t;
    ++launches;
    launched_frames += (int64_t)L->reqs.size();
    out.push_back(L);
    any = true;
  }
  return any;
}

// The device work of one launch (called without mu).
void mimo_server::run_launch(Launch* L) {
  hipStream_t st = streams[L->slot];
  for (Req* r : L->reqs)
    if (r->ready) (void)hipStreamWaitEvent(st, r->ready, 0);
  Req* f = L->reqs[0];
  int status = MIMO_OK;
  if (f->kind == 0 && f->up.sinr_mode != MIMO_SINR_APPROX) {
    const void* Y = f->up.Y;
    if (f->ch.dtype != MIMO_C32) {
      status = mimo_convert(f->up.Y, ptr(f->scratch_off), f->ch.dtype, f->ch.n_sc, f->ch.B, f->up.S, st);
      Y = ptr(f->scratch_off);
    }
    mimo_shape sh{f->ch.B, f->ch.U, f->up.S, f->up.K, f->ch.n_sc};
    void* out2 = f->up.want_xhat ? ptr(f->out_off + round_up(f->out_bytes)) : nullptr;
    if (status == MIMO_OK)
      status = mimo_detect_cg(&sh, f->ch.H, Y, f->ch.dtype, f->up.n0, f->up.es, f->up.qam_bits,
                              f->up.sinr_mode, f->up.scalar_prec, (float*)ptr(f->out_off), out2,
                              nullptr, nullptr, nullptr, 0, st);
  } else {
    mimo_frame frames[MIMO_MAX_BATCH];
    int n = 0;
    for (Req* r : L->reqs) {
      mimo_frame& fr = frames[n++];
      std::memset(&fr, 0, sizeof(fr));
      fr.n_sc = r->ch.n_sc;
      fr.B = r->ch.B;
      fr.U = r->ch.U;
      fr.S = r->S();
      fr.H = r->ch.H;
      fr.gram = frame_gram(r->ch);
      fr.out = ptr(r->out_off);
      if (r->kind == 0) {
        fr.K = r->up.K;
        fr.Y = r->up.Y;
        if (r->ch.dtype != MIMO_C32 && status == MIMO_OK) {
          status = mimo_convert(r->up.Y, ptr(r->scratch_off), r->ch.dtype, r->ch.n_sc, r->ch.B,
                                r->up.S, st);
          fr.Y = ptr(r->scratch_off);
        }
        fr.out2 = r->up.want_xhat ? ptr(r->out_off + round_up(r->out_bytes)) : nullptr;
        fr.n0 = r->up.n0;
        fr.es = r->up.es;
      } else {
        fr.K = r->dn.K;
        fr.Y = r->dn.T;
        fr.out2 = ptr(r->out_off + round_up(r->out_bytes));
        fr.beta = r->dn.beta;
        fr.normalize = r->dn.normalize;
      }
    }
    if (status == MIMO_OK)
      status = f->kind == 0
                   ? mimo_detect_cg_batch(frames, n, f->ch.dtype, f->up.qam_bits,
                                          f->up.scalar_prec, st)
                   : mimo_precode_cg_batch(frames, n, f->ch.dtype, f->dn.scalar_prec, st);
  }
  L->status = status;
  if (hipEventRecord(L->done, st) != hipSuccess && L->status == MIMO_OK) L->status = MIMO_EHIP;
}

void mimo_server::finish_locked(Launch* L, double t_done) {
  for (Req* r : L->reqs) {
    r->t_done = t_done;
    r->status = L->status;
    if (r->has_scratch) pool.release(r->scratch_off, r->scratch_bytes);
    r->has_scratch = false;
    if (r->ready) {
      spare_events.push_back(r->ready);
      r->ready = nullptr;
    }
    const int64_t solves = r->ch.n_sc * r->S();
    records.push_back(DoneRec{r->id, r->t_submit, t_done, solves,
                              r->kind == 0 ? solves * r->ch.U * r->up.qam_bits : 0});
    if (cfg.keep_outputs) {
      r->holders = 1;                     // the caller's, until mimo_server_release
      held[r->id] = r;
    } else {
      pool.release(r->out_off, r->out_bytes + r->out2_bytes);
      r->out_bytes = r->out2_bytes = 0;   // completion carries NULL outputs
    }
    completed.push_back(r);
  }
  spare_events.push_back(L->done);
  free_slots.push_back(L->slot);
  delete L;
}

void mimo_server::loop() {
  (void)hipSetDevice(device);
  std::vector<Launch*> todo, finished;
  std::vector<double> finished_t;
  for (;;) {
    todo.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      admit_locked(todo);
      if (todo.empty()) {
        if (!running && inflight.empty()) {
          // shutting down with nothing in flight: what is still queued can
          // never be admitted (outputs the caller holds fill the budget)
          for (Req* r : queue) {
            if (r->ready) spare_events.push_back(r->ready);
            delete r;
          }
          queue.clear();
          cv_done.notify_all();
          return;
        }
        if (inflight.empty()) {
          cv_work.wait(lk);
          continue;
        }
      }
    }
    for (Launch* L : todo) run_launch(L);
    finished.clear();
    finished_t.clear();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (Launch* L : todo) inflight.push_back(L);
    }
    // completions: query without the lock (HIP calls), then publish
    std::vector<Launch*> snapshot;
    {
      std::lock_guard<std::mutex> lk(mu);
      snapshot = inflight;
    }
    for (Launch* L : snapshot) {
      if (hipEventQuery(L->done) == hipSuccess) {
        float ms = 0.f;
        double t = now();
        if (hipEventElapsedTime(&ms, ref_event, L->done) == hipSuccess) t = t_ref + ms * 1e-3;
        finished.push_back(L);
        finished_t.push_back(t);
      }
    }
    if (!finished.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < finished.size(); ++i) {
        inflight.erase(std::find(inflight.begin(), inflight.end(), finished[i]));
        finish_locked(finished[i], finished_t[i]);
      }
      cv_done.notify_all();
    } else if (todo.empty()) {
      // launches in flight, nothing admitted: wait briefly for new work
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

namespace {

int validate_cfg(const mimo_server_config* c) {
  if (!c) return fail(MIMO_EINVAL, "config is NULL");
  if (c->hbm_budget <= 0) return fail(MIMO_EINVAL, "hbm_budget=%lld must be > 0", (long long)c->hbm_budget);
  if (c->n_slots < 1 || c->n_slots > MIMO_SERVE_MAX_SLOTS)
    return fail(MIMO_EINVAL, "n_slots=%d outside [1, %d]", c->n_slots, MIMO_SERVE_MAX_SLOTS);
  if (c->max_batch < 1 || c->max_batch > MIMO_MAX_BATCH)
    return fail(MIMO_EINVAL, "max_batch=%d outside [1, %d]", c->max_batch, MIMO_MAX_BATCH);
  if (c->lookahead < 1) return fail(MIMO_EINVAL, "lookahead=%d < 1", c->lookahead);
  return MIMO_OK;
}

struct DLCtx {
  DLManagedTensor t;
  int64_t shape[4];
  mimo_server* s;
  std::shared_ptr<std::atomic<bool>> alive;
  int64_t id;
};

void dl_deleter(DLManagedTensor* t) {
  DLCtx* c = (DLCtx*)t->manager_ctx;
  if (c->alive->load()) {
    mimo_server* s = c->s;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->held.find(c->id);
    if (it != s->held.end() && --it->second->holders == 0) {
      s->free_request_locked(it->second);
      s->held.erase(it);
      s->cv_work.notify_all();
    }
  }
  delete c;
}

int submit(mimo_server* s, Req* r, void* ready_stream, int64_t* req_id) {
  if (ready_stream) {
    hipEvent_t e = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      e = s->event_locked(0);
    }
    if (!e || hipEventRecord(e, (hipStream_t)ready_stream) != hipSuccess) {
      delete r;
      return fail(MIMO_EHIP, "recording the input event failed");
    }
    r->ready = e;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->running) {
    if (r->ready) s->spare_events.push_back(r->ready);
    delete r;
    return fail(MIMO_EINVAL, "server is shutting down");
  }
  r->id = s->next_id++;
  r->t_submit = s->now();
  r->key = batch_key(*r);
  s->queue.push_back(r);
  *req_id = r->id;
  s->cv_work.notify_all();
  return MIMO_OK;
}

int lookup_channel(mimo_server* s, int64_t ch_id, Channel* ch) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->channels.find(ch_id);
  if (it == s->channels.end()) return fail(MIMO_EINVAL, "channel %lld is not registered", (long long)ch_id);
  *ch = it->second;
  return MIMO_OK;
}

int check_fits(mimo_server* s, const Req& r) {
  std::lock_guard<std::mutex> lk(s->mu);
  if ((int64_t)r.need() + s->channel_bytes > s->cfg.hbm_budget)
    return fail(MIMO_EUNSUPPORTED, "request needs %zu bytes; budget %lld minus channels %lld",
                r.need(), (long long)s->cfg.hbm_budget, (long long)s->channel_bytes);
  return MIMO_OK;
}

}  // namespace

extern "C" {

int mimo_server_create(const mimo_server_config* cfg, int device, mimo_server** out) {
  mimo::set_last_error("");
  if (!out) return fail(MIMO_EINVAL, "out is NULL");
  *out = nullptr;
  const int st = validate_cfg(cfg);
  if (st != MIMO_OK) return st;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return fail(MIMO_EINVAL, "device %d unavailable", device);
  auto* s = new mimo_server;
  s->cfg = *cfg;
  s->device = device;
  s->paused = cfg->paused != 0;
  s->origin = std::chrono::steady_clock::now();
  hipError_t e = hipMalloc((void**)&s->pool_base, (size_t)cfg->hbm_budget);
  for (int i = 0; e == hipSuccess && i < cfg->n_slots; ++i) {
    e = hipStreamCreate(&s->streams[i]);      // default priority
    s->free_slots.push_back(cfg->n_slots - 1 - i);
  }
  if (e == hipSuccess) e = hipEventCreate(&s->ref_event);
  if (e == hipSuccess) {
    // host time of the reference event: tightest of several round trips
    double best = 1e30;
    for (int i = 0; i < 20 && e == hipSuccess; ++i) {
      hipEvent_t ev = nullptr;
      e = hipEventCreate(&ev);
      if (e != hipSuccess) break;
      const double ta = s->now();
      e = hipEventRecord(ev, s->streams[0]);
      if (e == hipSuccess) e = hipEventSynchronize(ev);
      const double tb = s->now();
      if (e == hipSuccess && tb - ta < best) {
        best = tb - ta;
        std::swap(ev, s->ref_event);
        s->t_ref = 0.5 * (ta + tb);
      }
      (void)hipEventDestroy(ev);
    }
  }
  if (e != hipSuccess) {
    const char* msg = hipGetErrorString(e);
    for (int i = 0; i < cfg->n_slots; ++i)
      if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
    if (s->pool_base) (void)hipFree(s->pool_base);
    delete s;
    (void)hipSetDevice(prev);
    return fail(MIMO_EHIP, "server setup: %s", msg);
  }
  s->pool.init((size_t)cfg->hbm_budget);
  s->thread = std::thread([s] { s->loop(); });
  (void)hipSetDevice(prev);
  *out = s;
  return MIMO_OK;
}

int mimo_server_destroy(mimo_server* s) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = false;
    s->running = false;
    s->cv_work.notify_all();
  }
  s->thread.join();
  s->alive->store(false);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (Req* r : s->completed)
    if (!s->held.count(r->id)) delete r;
  for (auto& kv : s->held) delete kv.second;
  for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
  (void)hipEventDestroy(s->ref_event);
  for (int i = 0; i < s->cfg.n_slots; ++i) (void)hipStreamDestroy(s->streams[i]);
  (void)hipFree(s->pool_base);
  (void)hipSetDevice(prev);
  delete s;
  return MIMO_OK;
}

int mimo_server_register_channel(mimo_server* s, int64_t ch_id, const void* H, int in_dtype,
                                 int64_t n_sc, int32_t B, int32_t U) {
  return mimo_server_register_channel_gram(s, ch_id, H, nullptr, in_dtype, n_sc, B, U);
}

int mimo_server_register_channel_gram(mimo_server* s, int64_t ch_id, const void* H,
                                      const void* G, int in_dtype, int64_t n_sc, int32_t B,
                                      int32_t U) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  if (!H || ((uintptr_t)H & 15u)) return fail(MIMO_EINVAL, "H is NULL or not 16-byte aligned");
  if ((uintptr_t)G & 7u) return fail(MIMO_EINVAL, "G is not 8-byte aligned");
  if (in_dtype != MIMO_C32 && in_dtype != MIMO_C16 && in_dtype != MIMO_CBF16)
    return fail(MIMO_EINVAL, "in_dtype=%d unknown", in_dtype);
  if (U > MIMO_MAX_USERS_COMMON && U <= B && B <= MIMO_MAX_ANTENNAS)
    return fail(MIMO_EUNSUPPORTED, "U=%d > %d", U, MIMO_MAX_USERS_COMMON);
  if (n_sc < 1 || U < 1 || U > MIMO_MAX_USERS_COMMON || B < U || B > MIMO_MAX_ANTENNAS ||
      (in_dtype != MIMO_C32 && B % 8))
    return fail(MIMO_EINVAL, "bad channel shape n_sc=%lld B=%d U=%d", (long long)n_sc, B, U);
  const int64_t bytes = n_sc * B * U * (in_dtype == MIMO_C32 ? 8 : 4) + (G ? n_sc * U * U * 8 : 0);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->channels.find(ch_id);
  const int64_t old = it == s->channels.end() ? 0 : it->second.bytes;
  if (s->channel_bytes - old + bytes + (int64_t)s->pool.used() > s->cfg.hbm_budget)
    return fail(MIMO_EUNSUPPORTED, "channel %lld (%lld bytes) exceeds the HBM budget",
                (long long)ch_id, (long long)bytes);
  s->channels[ch_id] = Channel{H, in_dtype, n_sc, B, U, bytes, G};
  s->channel_bytes += bytes - old;
  return MIMO_OK;
}

int mimo_server_unregister_channel(mimo_server* s, int64_t ch_id) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->channels.find(ch_id);
  if (it == s->channels.end()) return fail(MIMO_EINVAL, "channel %lld is not registered", (long long)ch_id);
  s->channel_bytes -= it->second.bytes;
  s->channels.erase(it);
  s->cv_work.notify_all();
  return MIMO_OK;
}

int mimo_server_submit_uplink(mimo_server* s, const mimo_uplink_req* q, void* ready_stream,
                              int64_t* req_id) {
  mimo::set_last_error("");
  if (!s || !q || !req_id) return fail(MIMO_EINVAL, "NULL argument");
  Channel ch;
  int st = lookup_channel(s, q->ch_id, &ch);
  if (st != MIMO_OK) return st;
  if (!q->Y || ((uintptr_t)q->Y & 15u)) return fail(MIMO_EINVAL, "Y is NULL or not 16-byte aligned");
  if (q->S < 1 || q->K < 1 || q->K > 1024) return fail(MIMO_EINVAL, "S=%d K=%d", q->S, q->K);
  if (q->qam_bits != 2 && q->qam_bits != 4 && q->qam_bits != 6 && q->qam_bits != 8)
    return fail(MIMO_EUNSUPPORTED, "qam_bits=%d not in {2,4,6,8}", q->qam_bits);
  if (q->sinr_mode != MIMO_SINR_APPROX && q->sinr_mode != MIMO_SINR_EXACT)
    return fail(MIMO_EINVAL, "sinr_mode=%d unknown", q->sinr_mode);
  if (q->scalar_prec != MIMO_SCALAR_F32 && q->scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", q->scalar_prec);
  if (!(q->n0 > 0.f) || !(q->es > 0.f)) return fail(MIMO_EINVAL, "n0 and es must be > 0");
  const int64_t span = (int64_t)q->S * 8 * std::max<int64_t>(ch.B, 4 * ch.U);
  if (span >= MIMO_MAX_SPAN_BYTES) return fail(MIMO_EUNSUPPORTED, "S=%d too large", q->S);
  Req* r = new Req;
  r->kind = 0;
  r->up = *q;
  r->ch = ch;
  r->out_bytes = (size_t)ch.n_sc * ch.U * q->S * q->qam_bits * 4;
  r->out2_bytes = q->want_xhat ? (size_t)ch.n_sc * ch.U * q->S * 8 : 0;
  r->has_scratch = ch.dtype != MIMO_C32;
  r->scratch_bytes = r->has_scratch ? (size_t)ch.n_sc * ch.B * q->S * 4 : 0;
  if ((st = check_fits(s, *r)) != MIMO_OK) {
    delete r;
    return st;
  }
  return submit(s, r, ready_stream, req_id);
}

int mimo_server_submit_downlink(mimo_server* s, const mimo_downlink_req* q, void* ready_stream,
                                int64_t* req_id) {
  mimo::set_last_error("");
  if (!s || !q || !req_id) return fail(MIMO_EINVAL, "NULL argument");
  Channel ch;
  int st = lookup_channel(s, q->ch_id, &ch);
  if (st != MIMO_OK) return st;
  if (!q->T || ((uintptr_t)q->T & 15u)) return fail(MIMO_EINVAL, "T is NULL or not 16-byte aligned");
  if (q->S < 1 || q->K < 1 || q->K > 1024) return fail(MIMO_EINVAL, "S=%d K=%d", q->S, q->K);
  if (q->scalar_prec != MIMO_SCALAR_F32 && q->scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", q->scalar_prec);
  if (!(q->beta >= 0.f)) return fail(MIMO_EINVAL, "beta must be >= 0");
  const int64_t span = (int64_t)q->S * 8 * std::max<int64_t>(ch.B, 4 * ch.U);
  if (span >= MIMO_MAX_SPAN_BYTES) return fail(MIMO_EUNSUPPORTED, "S=%d too large", q->S);
  Req* r = new Req;
  r->kind = 1;
  r->dn = *q;
  r->ch = ch;
  r->out_bytes = (size_t)ch.n_sc * ch.B * q->S * 8;
  r->out2_bytes = (size_t)ch.n_sc * q->S * 4;
  if ((st = check_fits(s, *r)) != MIMO_OK) {
    delete r;
    return st;
  }
  return submit(s, r, ready_stream, req_id);
}

int mimo_server_poll(mimo_server* s, mimo_completion* out, int max, int64_t timeout_us) {
  mimo::set_last_error("");
  if (!s || (!out && max > 0)) return fail(MIMO_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->completed.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [s] { return !s->completed.empty(); });
  int n = 0;
  while (n < max && !s->completed.empty()) {
    Req* r = s->completed.front();
    s->completed.pop_front();
    mimo_completion& c = out[n++];
    c.req_id = r->id;
    c.status = r->status;
    c.kind = r->kind;
    c.t_submit = r->t_submit;
    c.t_admit = r->t_admit;
    c.t_done = r->t_done;
    const bool kept = s->cfg.keep_outputs != 0;
    c.out = kept ? s->ptr(r->out_off) : nullptr;
    c.out2 = kept && r->out2_bytes ? s->ptr(r->out_off + round_up(r->out_bytes)) : nullptr;
    c.n_sc = r->ch.n_sc;
    c.B = r->ch.B;
    c.U = r->ch.U;
    c.S = r->S();
    c.qam_bits = r->kind == 0 ? r->up.qam_bits : 0;
    c.solves = r->ch.n_sc * r->S();
    c.llr_bits = r->kind == 0 ? c.solves * r->ch.U * r->up.qam_bits : 0;
    if (!kept) delete r;                  // nothing left to release
  }
  return n;
}

int mimo_server_release(mimo_server* s, int64_t req_id) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->held.find(req_id);
  if (it == s->held.end()) return fail(MIMO_EINVAL, "request %lld holds no outputs", (long long)req_id);
  if (--it->second->holders == 0) {
    s->free_request_locked(it->second);
    s->held.erase(it);
    s->cv_work.notify_all();
  }
  return MIMO_OK;
}

int mimo_server_dlpack(mimo_server* s, int64_t req_id, int which, void** managed) {
  mimo::set_last_error("");
  if (!s || !managed || (which != 0 && which != 1)) return fail(MIMO_EINVAL, "bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->held.find(req_id);
  if (it == s->held.end()) return fail(MIMO_EINVAL, "request %lld holds no outputs", (long long)req_id);
  Req* r = it->second;
  if (which == 1 && r->out2_bytes == 0) return fail(MIMO_EINVAL, "request has no second output");
  DLCtx* c = new DLCtx;
  c->s = s;
  c->alive = s->alive;
  c->id = req_id;
  DLTensor& t = c->t.dl_tensor;
  std::memset(&t, 0, sizeof(t));
  t.data = s->ptr(r->out_off + (which ? round_up(r->out_bytes) : 0));
  t.device = DLDevice{kDLROCM, s->device};
  t.shape = c->shape;
  const int64_t n = r->ch.n_sc, S = r->S();
  if (r->kind == 0 && which == 0) {           // llr [n][U][S][m]
    t.ndim = 4;
    t.dtype = DLDataType{kDLFloat, 32, 1};
    c->shape[0] = n; c->shape[1] = r->ch.U; c->shape[2] = S; c->shape[3] = r->up.qam_bits;
  } else if (r->kind == 0) {                  // xhat [n][U][S]
    t.ndim = 3;
    t.dtype = DLDataType{kDLComplex, 64, 1};
    c->shape[0] = n; c->shape[1] = r->ch.U; c->shape[2] = S;
  } else if (which == 0) {                    // Q [n][B][S]
    t.ndim = 3;
    t.dtype = DLDataType{kDLComplex, 64, 1};
    c->shape[0] = n; c->shape[1] = r->ch.B; c->shape[2] = S;
  } else {                                    // qnorm [n][S]
    t.ndim = 2;
    t.dtype = DLDataType{kDLFloat, 32, 1};
    c->shape[0] = n; c->shape[1] = S;
  }
  t.strides = nullptr;                        // compact row-major
  c->t.manager_ctx = c;
  c->t.deleter = dl_deleter;
  ++r->holders;
  *managed = &c->t;
  return MIMO_OK;
}

int mimo_server_pause(mimo_server* s) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->paused = true;
  s->t_resume = -1;
  return MIMO_OK;
}

int mimo_server_resume(mimo_server* s) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->paused) {
    s->paused = false;
    s->t_resume = s->now();
    s->cv_work.notify_all();
  }
  return MIMO_OK;
}

int mimo_server_drain(mimo_server* s, int64_t timeout_us) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto idle = [s] { return s->queue.empty() && s->inflight.empty(); };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, idle);
    return MIMO_OK;
  }
  if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), idle))
    return fail(MIMO_EINVAL, "queue did not drain in %lld us", (long long)timeout_us);
  return MIMO_OK;
}

int mimo_server_stats_get(mimo_server* s, int64_t skip, int reset, mimo_server_stats* out) {
  mimo::set_last_error("");
  if (!s || !out) return fail(MIMO_EINVAL, "NULL argument");
  std::vector<DoneRec> recs;
  double t_rel;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    recs = s->records;
    t_rel = s->t_resume;
    out->peak_bytes = s->peak_bytes;
    out->budget_waits = s->budget_waits;
    out->launches = s->launches;
    out->mean_batch = s->launches ? (double)s->launched_frames / s->launches : 0.0;
    if (reset) s->records.clear();
  }
  std::sort(recs.begin(), recs.end(),
            [](const DoneRec& a, const DoneRec& b) { return a.t_submit < b.t_submit; });
  if (skip > 0) recs.erase(recs.begin(), recs.begin() + std::min<size_t>(recs.size(), (size_t)skip));
  out->frames = (int64_t)recs.size();
  if (recs.empty()) {
    out->p50_ms = out->p99_ms = out->mean_ms = 0;
    out->frames_per_s = out->solves_per_s = out->llr_gbit_s = 0;
    return MIMO_OK;
  }
  std::vector<double> lat;
  lat.reserve(recs.size());
  double t0 = 1e300, t1 = -1e300, sum = 0;
  int64_t solves = 0, bits = 0;
  for (const DoneRec& d : recs) {
    const double arrive = t_rel >= 0 ? std::max(d.t_submit, t_rel) : d.t_submit;
    lat.push_back(d.t_done - arrive);
    sum += d.t_done - arrive;
    t0 = std::min(t0, arrive);
    t1 = std::max(t1, d.t_done);
    solves += d.solves;
    bits += d.llr_bits;
  }
  auto pct = [&](double q) {   // linear interpolation between order statistics
    std::vector<double> v = lat;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
  };
  const double span = std::max(t1 - t0, 1e-12);
  out->p50_ms = pct(0.50) * 1e3;
  out->p99_ms = pct(0.99) * 1e3;
  out->mean_ms = sum / (double)lat.size() * 1e3;
  out->frames_per_s = (double)recs.size() / span;
  out->solves_per_s = (double)solves / span;
  out->llr_gbit_s = (double)bits / span / 1e9;
  return MIMO_OK;
}

int mimo_server_memory(mimo_server* s, int64_t* channel_bytes, int64_t* pool_bytes) {
  mimo::set_last_error("");
  if (!s) return fail(MIMO_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (channel_bytes) *channel_bytes = s->channel_bytes;
  if (pool_bytes) *pool_bytes = (int64_t)s->pool.used();
  return MIMO_OK;
}

}  // extern "C"
