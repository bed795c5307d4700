// Continuous batching of independent imaging requests (clsimg_server_*).
//
// Requests for arrays of up to 48 antennas live on the device in slots: each
// owns a slice of one HBM arena (steering tables, data matrix, lists, outer
// state) and advances by one Table I step per launch of the batched outer-step
// kernel, one workgroup per request; one launch of the batched multiplier
// kernel serves all of them.  Slots are grouped by the array's tile count, one
// launch pair per group and step.  Between rounds of steps the host reads the
// small outer states back, retires finished requests and admits waiting ones
// into the freed slots and arena space, so new work joins work already on the
// GPU.  Requests the device loop cannot hold (more antennas, or a free set
// beyond its on-chip capacity) are solved by worker threads, each with its own
// context and stream, overlapping with the batch and each other on the device.
//
// Every request computes exactly what clsimg_solve computes for it alone: the
// same set-up launches, the same outer-step and multiplier code, and the same
// multiplier block partition (blocks of one request never depend on others).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/clsimg.h"
#include "kernels.h"
#include "request.h"

using namespace clsimg;

namespace {

constexpr int kMaxSlots = 1024;     // one workgroup per slot and step
constexpr int kKeysPerReq = 2048;   // multiplier blocks of the largest grid
constexpr int kMaxWorkers = 8;      // threads (contexts, streams) for the other requests
constexpr size_t kAlign = 256;

struct Job {
  int64_t ticket;
  clsimg_request* req;
};

struct Slot {
  Job job;
  size_t off = 0, bytes = 0;  // arena slice
  ReqLayout L;
  OuterParams op;
  BeamLamItem it;
  int mt = 0;
};

// first-fit allocator over one device arena
struct Arena {
  char* base = nullptr;
  size_t bytes = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> size, coalesced
  void reset(char* b, size_t n) {
    base = b;
    bytes = n;
    free_.clear();
    free_[0] = n;
  }
  bool take(size_t n, size_t& off) {
    n = (n + kAlign - 1) & ~(kAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      off = it->first;
      const size_t rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used += n;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t n) {
    n = (n + kAlign - 1) & ~(kAlign - 1);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct clsimg_server {
  int device = 0;
  clsimg_opts opts{};
  int max_slots = 0;
  int steps_per_poll = 16;
  clsimg_ctx* ctx = nullptr;  // set-up scratch of the batch
  hipStream_t stream = nullptr;
  Arena arena;
  void* d_params = nullptr;  // OuterParams[max_slots] then BeamLamItem[max_slots]
  char* h_stage = nullptr;   // pinned: parameter upload and state read-back
  std::deque<Job> pending;
  std::vector<Slot> slots;
  bool params_dirty = true;
  struct Group {
    int mt, first, n, P, bpr;
  };
  std::vector<Group> groups;
  int64_t next_ticket = 1, submitted = 0, admitted = 0, completed = 0, steps = 0;
  // workers for requests outside the device loop: one context and stream each
  std::vector<clsimg_ctx*> wctx;
  std::vector<hipStream_t> wstream;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> large_q;  // guarded by mu
  int large_active = 0;     // guarded by mu: jobs being solved by workers
  bool stop = false;        // guarded by mu
  std::deque<int64_t> done;  // guarded by mu
};

namespace {

struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void worker_main(clsimg_server* s, int w) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->large_q.empty(); });
      if (s->stop) return;
      j = s->large_q.front();
      s->large_q.pop_front();
      ++s->large_active;
    }
    clsimg_request& q = *j.req;
    int st = clsimg_solve(s->wctx[w], q.R, &q.array, &q.grid, q.noise_diag, &s->opts, nullptr, nullptr, q.sigma,
                          q.state, q.mf, q.gamma, &q.stats, s->wstream[w]);
    if (hipStreamSynchronize(s->wstream[w]) != hipSuccess && st >= 0) st = CLSIMG_EHIP;
    q.stats.status = st;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      --s->large_active;
      s->done.push_back(j.ticket);
    }
    s->cv_done.notify_all();
  }
}

void to_worker(clsimg_server* s, const Job& j) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->large_q.push_back(j);
  }
  s->cv_work.notify_one();
}

void finish_now(clsimg_server* s, const Job& j, int status) {
  j.req->stats.status = status;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(j.ticket);
  }
}

ReqLayout layout_for(const clsimg_server* s, const clsimg_request& q) {
  ReqLayout L = request_layout(q.array.P, q.grid.nl, q.grid.nm, s->opts.cost == CLSIMG_COST_PWLS, kKeysPerReq);
  L.tiles = beam_batch_tiles(s->max_slots, q.grid.nl * q.grid.nm);  // as if every slot were busy
  return L;
}

// Admit waiting requests into free slots while the arena has room for them.
int admit(clsimg_server* s) {
  for (auto it = s->pending.begin(); it != s->pending.end() && (int)s->slots.size() < s->max_slots;) {
    clsimg_request& q = *it->req;
    Slot sl;
    sl.job = *it;
    sl.L = layout_for(s, q);
    if (!s->arena.take(sl.L.bytes, sl.off)) {
      ++it;  // a smaller request further back may still fit
      continue;
    }
    sl.bytes = sl.L.bytes;
    sl.mt = pad_p(q.array.P) / 8;
    // the set-up may grow the context's scratch, which the previous request's
    // set-up may still be using on the stream
    if (hipStreamSynchronize(s->stream) != hipSuccess) return CLSIMG_EHIP;
    const int st = request_setup(s->ctx, q, &s->opts, s->arena.base + sl.off, sl.L, sl.op, sl.it, s->stream);
    it = s->pending.erase(it);
    if (st != CLSIMG_OK) {  // e.g. a covariance that is not positive definite
      (void)hipStreamSynchronize(s->stream);
      s->arena.give(sl.off, sl.bytes);
      finish_now(s, sl.job, st);
      continue;
    }
    ++s->admitted;
    s->slots.push_back(sl);
    s->params_dirty = true;
  }
  return CLSIMG_OK;
}

// Slots sorted by tile count; parameters of each group contiguous on the device.
int upload_params(clsimg_server* s) {
  std::stable_sort(s->slots.begin(), s->slots.end(), [](const Slot& a, const Slot& b) { return a.mt < b.mt; });
  const int n = (int)s->slots.size();
  OuterParams* hp = reinterpret_cast<OuterParams*>(s->h_stage);
  BeamLamItem* hi = reinterpret_cast<BeamLamItem*>(s->h_stage + (size_t)s->max_slots * sizeof(OuterParams));
  s->groups.clear();
  for (int i = 0; i < n; ++i) {
    const Slot& sl = s->slots[i];
    hp[i] = sl.op;
    hi[i] = sl.it;
    if (s->groups.empty() || s->groups.back().mt != sl.mt)
      s->groups.push_back({sl.mt, i, 0, sl.op.P, 1});
    auto& g = s->groups.back();
    ++g.n;
    g.bpr = std::max(g.bpr, sl.it.nblk);
  }
  char* dp = static_cast<char*>(s->d_params);
  if (hipMemcpyAsync(dp, hp, (size_t)n * sizeof(OuterParams), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipMemcpyAsync(dp + (size_t)s->max_slots * sizeof(OuterParams), hi, (size_t)n * sizeof(BeamLamItem),
                     hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)  // the staging is reused for read-backs
    return CLSIMG_EHIP;
  s->params_dirty = false;
  return CLSIMG_OK;
}

int run_round(clsimg_server* s) {
  char* dp = static_cast<char*>(s->d_params);
  const OuterParams* op = reinterpret_cast<const OuterParams*>(dp);
  const BeamLamItem* it = reinterpret_cast<const BeamLamItem*>(dp + (size_t)s->max_slots * sizeof(OuterParams));
  for (int b = 0; b < s->steps_per_poll; ++b) {
    for (const auto& g : s->groups) {
      if (launch_outer_step_batch(op + g.first, g.n, g.P, s->stream) != hipSuccess) return CLSIMG_EHIP;
      if (launch_beam_lambda_batch(it + g.first, g.n, g.bpr, g.P, s->stream) != hipSuccess) return CLSIMG_EHIP;
    }
    ++s->steps;
  }
  // read back the outer states and retire the finished requests
  OuterState* hs = reinterpret_cast<OuterState*>(s->h_stage);
  const int n = (int)s->slots.size();
  for (int i = 0; i < n; ++i)
    if (hipMemcpyAsync(hs + i, s->slots[i].op.st, sizeof(OuterState), hipMemcpyDeviceToHost, s->stream) !=
        hipSuccess)
      return CLSIMG_EHIP;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return CLSIMG_EHIP;
  std::vector<Slot> keep;
  std::vector<std::pair<Job, int>> fin;
  keep.reserve(n);
  for (int i = 0; i < n; ++i) {
    Slot& sl = s->slots[i];
    const OuterState& S = hs[i];
    if (!S.done) {
      keep.push_back(sl);
      continue;
    }
    if (S.fallback) {
      // beyond the on-chip capacity: the worker solves it as clsimg_solve would
      s->arena.give(sl.off, sl.bytes);
      to_worker(s, sl.job);
      continue;
    }
    const int st = request_finish(*sl.job.req, &s->opts, s->arena.base + sl.off, sl.L, S, s->stream);
    fin.push_back({sl.job, st});
    s->arena.give(sl.off, sl.bytes);  // stream-ordered: the next use is enqueued after the finish
  }
  if (!fin.empty() && hipStreamSynchronize(s->stream) != hipSuccess) return CLSIMG_EHIP;
  for (auto& f : fin) finish_now(s, f.first, f.second);
  if ((int)keep.size() != n) s->params_dirty = true;
  s->slots.swap(keep);
  return CLSIMG_OK;
}

int take_done(clsimg_server* s, int64_t* tickets, int32_t cap, int32_t* n_done) {
  std::lock_guard<std::mutex> lk(s->mu);
  int k = 0;
  while (k < cap && !s->done.empty()) {
    tickets[k++] = s->done.front();
    s->done.pop_front();
  }
  s->completed += k;
  *n_done = k;
  return CLSIMG_OK;
}

}  // namespace

extern "C" {

int clsimg_server_create(clsimg_server** out, int32_t device, int32_t max_slots, size_t hbm_budget_bytes,
                         int32_t steps_per_poll, int32_t workers, const clsimg_opts* o) {
  if (!out) return CLSIMG_EINVAL;
  *out = nullptr;
  if (!o || max_slots < 1 || max_slots > kMaxSlots || steps_per_poll < 1 || steps_per_poll > 1024 ||
      workers < 1 || workers > kMaxWorkers)
    return CLSIMG_EINVAL;
  if (o->cost != CLSIMG_COST_LS && o->cost != CLSIMG_COST_PWLS) return CLSIMG_EINVAL;
  if (o->nsamples <= 0 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CLSIMG_EINVAL;
  DeviceScope scope(device);
  clsimg_server* s = new clsimg_server();
  s->device = device;
  s->opts = *o;
  s->max_slots = max_slots;
  s->steps_per_poll = steps_per_poll;
  const size_t arena = hbm_budget_bytes ? hbm_budget_bytes : (size_t)1 << 30;
  void* base = nullptr;
  int st = clsimg_create(&s->ctx, device, 0);
  if (st == CLSIMG_OK && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) st = CLSIMG_EHIP;
  for (int w = 0; w < workers && st == CLSIMG_OK; ++w) {
    clsimg_ctx* c = nullptr;
    hipStream_t ws = nullptr;
    st = clsimg_create(&c, device, 0);
    if (st == CLSIMG_OK) s->wctx.push_back(c);
    if (st == CLSIMG_OK && hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) st = CLSIMG_EHIP;
    if (st == CLSIMG_OK) s->wstream.push_back(ws);
  }
  if (st == CLSIMG_OK && hipMalloc(&base, arena) != hipSuccess) st = CLSIMG_ENOMEM;
  if (st == CLSIMG_OK) s->arena.reset(static_cast<char*>(base), arena);
  const size_t pbytes = (size_t)max_slots * (sizeof(OuterParams) + sizeof(BeamLamItem));
  const size_t hbytes = std::max(pbytes, (size_t)max_slots * sizeof(OuterState));
  if (st == CLSIMG_OK && hipMalloc(&s->d_params, pbytes) != hipSuccess) st = CLSIMG_ENOMEM;
  if (st == CLSIMG_OK && hipHostMalloc((void**)&s->h_stage, hbytes, hipHostMallocDefault) != hipSuccess)
    st = CLSIMG_ENOMEM;
  if (st != CLSIMG_OK) {
    clsimg_server_destroy(s);
    return st;
  }
  for (int w = 0; w < workers; ++w) s->workers.emplace_back(worker_main, s, w);
  *out = s;
  return CLSIMG_OK;
}

int clsimg_server_destroy(clsimg_server* s) {
  if (!s) return CLSIMG_EINVAL;
  DeviceScope scope(s->device);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();  // solves in progress are finished first
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto ws : s->wstream) (void)hipStreamSynchronize(ws);
  if (s->arena.base) (void)hipFree(s->arena.base);
  if (s->d_params) (void)hipFree(s->d_params);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->ctx) clsimg_destroy(s->ctx);
  for (auto c : s->wctx) clsimg_destroy(c);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  for (auto ws : s->wstream) (void)hipStreamDestroy(ws);
  delete s;
  return CLSIMG_OK;
}

int clsimg_server_submit(clsimg_server* s, clsimg_request* q, int64_t* ticket) {
  if (!s || !q || !ticket) return CLSIMG_EINVAL;
  *ticket = 0;
  if (!q->R || !q->sigma || !q->state) return CLSIMG_EINVAL;
  const clsimg_array* a = &q->array;
  const clsimg_grid* g = &q->grid;
  if (!a->pos_xy || a->P < 1 || a->P > CLSIMG_MAX_P || !(a->lambda > 0.0) || g->nl < 1 || g->nm < 1 ||
      (int64_t)g->nl * g->nm > CLSIMG_MAX_Q)
    return CLSIMG_EINVAL;
  const bool pwls = s->opts.cost == CLSIMG_COST_PWLS;
  if (s->opts.nsamples <= a->P + 1 && pwls && s->opts.kappa_d != 0.0) return CLSIMG_EINVAL;
  memset(&q->stats, 0, sizeof(q->stats));
  const Job j{s->next_ticket++, q};
  ++s->submitted;
  const int Q = g->nl * g->nm;
  const bool device = request_on_device(a->P) && beam_grid(Q) <= kKeysPerReq &&
                      layout_for(s, *q).bytes <= s->arena.bytes;
  if (!device) {
    to_worker(s, j);  // clsimg_solve on a worker (PWLS up to 96 antennas, else CLSIMG_ENOTSUP)
  } else {
    s->pending.push_back(j);
  }
  *ticket = j.ticket;
  return CLSIMG_OK;
}

int clsimg_server_poll(clsimg_server* s, int32_t wait, int64_t* tickets, int32_t cap, int32_t* n_done) {
  if (!s || !n_done || cap < 0 || (cap > 0 && !tickets)) return CLSIMG_EINVAL;
  *n_done = 0;
  DeviceScope scope(s->device);
  for (;;) {
    int st = admit(s);
    if (st != CLSIMG_OK) return st;
    if (!s->slots.empty()) {
      if (s->params_dirty && (st = upload_params(s)) != CLSIMG_OK) return st;
      if ((st = run_round(s)) != CLSIMG_OK) return st;
    }
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!wait || !s->done.empty()) break;
      if (s->pending.empty() && s->slots.empty()) {
        if (s->large_q.empty() && s->large_active == 0) break;  // nothing left to wait for
        // only the worker has work: sleep until it reports
        s->cv_done.wait(lk, [&] { return !s->done.empty(); });
        break;
      }
    }
  }
  return take_done(s, tickets, cap, n_done);
}

int clsimg_server_query(clsimg_server* s, clsimg_server_info* info) {
  if (!s || !info) return CLSIMG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  info->pending = (int32_t)s->pending.size();
  info->active = (int32_t)s->slots.size();
  info->worker_queued = (int32_t)s->large_q.size() + s->large_active;
  info->ready = (int32_t)s->done.size();
  info->submitted = s->submitted;
  info->completed = s->completed;
  info->admitted = s->admitted;
  info->step_rounds = s->steps;
  info->arena_bytes = s->arena.bytes;
  info->arena_used = s->arena.used;
  info->arena_peak = s->arena.peak;
  return CLSIMG_OK;
}

}  // extern "C"
