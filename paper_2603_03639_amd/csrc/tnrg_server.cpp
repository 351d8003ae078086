// Serving runtime of libtnrg: continuous batching of fidelity+gradient
// requests on one GPU (declarations and contract in tnrg.h).
//
// Each admitted request is one persistent grape_fidelity_grad launch on one
// of the server's streams, followed by an asynchronous copy of its
// per-trajectory flags into pinned host memory and an event.  progress()
// polls the events without blocking: a finished request either completes or,
// when a bond outgrew its capacity bucket, goes back to the head of the queue
// with the next bucket.  Workspaces are carved first-fit out of the caller's
// device arena, so admission is by HBM footprint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "tnrg.h"

int tnrg_set_error(int code, const char* msg);

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

int err(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return tnrg_set_error(code, buf);
}

// First-fit allocator over [0, size) in 256-byte granules; free blocks are
// kept sorted by offset and merged with their neighbours on release.
class Arena {
 public:
  Arena(char* base, size_t size) : base_(base), size_(size & ~(size_t)255) {
    if (size_) free_[0] = size_;
  }
  char* alloc(size_t n) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used_[off] = n;
      return base_ + off;
    }
    return nullptr;
  }
  void release(char* p) {
    auto u = used_.find((size_t)(p - base_));
    if (u == used_.end()) return;
    size_t off = u->first, n = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  size_t size() const { return size_; }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& f : free_) s += f.second;
    return s;
  }
  size_t largest_free() const {
    size_t s = 0;
    for (auto& f : free_) s = f.second > s ? f.second : s;
    return s;
  }

 private:
  char* base_;
  size_t size_;
  std::map<size_t, size_t> free_, used_;
};

struct Job {
  int64_t ticket = 0;
  tnrg_request req{};
  tnrg_model model{};
  std::vector<uint8_t> zz, xt;
  tnrg_mps_batch in{}, tg{};
  std::vector<int> buckets;  // capacities to try, in order
  size_t bucket = 0;         // index into buckets
  int launches = 0;
  int bypassed = 0;
  bool admitted_once = false;
  Clock::time_point t_submit, t_admit;
  char* ws = nullptr;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t* host_flags = nullptr;  // pinned
  size_t flags_cap = 0;
  std::unique_ptr<Job> job;
};

using PlanKey = std::tuple<int, int, int, int, int, int>;  // N, M, chi, xt_model, K, R

// The capacity-bucket plan: the last bucket that held every bond of a request
// of this shape, shared by all servers of the process.
std::mutex g_plan_mu;
std::map<PlanKey, int> g_plan;

int plan_get(const PlanKey& k) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plan.find(k);
  return it == g_plan.end() ? 0 : it->second;
}
void plan_put(const PlanKey& k, int cap) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plan[k] = cap;
}

// Buckets to try: 4, 8, ... below min(chi, 2^(N/2)), then that value, all
// at most max_dcap, starting from the plan's bucket `start` when there is one.
// floor: no bucket below the capacity of the request's input and target
// batches (the states hold them before their first truncation to chi).
std::vector<int> bucket_sequence(const tnrg_model& md, int start, int max_dcap, int floor) {
  const int half = md.n / 2;
  int cap_max = md.chi;
  if (half < 30 && (1 << half) < cap_max) cap_max = 1 << half;
  if (cap_max < floor) cap_max = floor;
  std::vector<int> seq;
  for (int b : {4, 8, 16, 32, 64, 128})
    if (b >= floor && b < cap_max && b <= max_dcap) seq.push_back(b);
  if (cap_max <= max_dcap) seq.push_back(cap_max);
  if (seq.empty()) seq.push_back(max_dcap < cap_max ? max_dcap : cap_max);
  if (start > 0) {
    std::vector<int> tail;
    for (int b : seq)
      if (b >= start) tail.push_back(b);
    if (tail.empty()) tail.push_back(seq.back());
    seq.swap(tail);
  }
  return seq;
}

}  // namespace

struct tnrg_server {
  explicit tnrg_server(char* base, size_t bytes) : arena(base, bytes) {}
  Arena arena;
  std::vector<Slot> slots;
  std::deque<std::unique_ptr<Job>> queue;
  std::deque<tnrg_completion> finished;
  int max_bypass = 0;
  int max_dcap = 0;  // largest capacity bucket a request may use
  int64_t next_ticket = 1;
  int64_t submitted = 0, admitted = 0, completed = 0, regrown = 0, cancelled = 0;
};

namespace {

void complete(tnrg_server* s, std::unique_ptr<Job> job, int status) {
  const auto now = Clock::now();
  tnrg_completion c{};
  c.ticket = job->ticket;
  c.status = status;
  c.dcap = job->buckets.empty() ? 0 : job->buckets[std::min(job->bucket, job->buckets.size() - 1)];
  c.launches = job->launches;
  c.queue_ms = job->admitted_once ? ms_between(job->t_submit, job->t_admit) : ms_between(job->t_submit, now);
  c.total_ms = ms_between(job->t_submit, now);
  s->finished.push_back(c);
  s->completed += 1;
}

// Launch `job` on slot `si` with its workspace already carved; returns the
// launch status (the job stays with the caller on failure).
int launch(tnrg_server* s, int si, Job* job, size_t ws_bytes) {
  Slot& sl = s->slots[si];
  const int cap = job->buckets[job->bucket];
  const tnrg_request& q = job->req;
  int rc = grape_fidelity_grad(&job->model, q.ux, q.uy, q.uzz, q.K, q.J, q.R, &job->in, &job->tg,
                               cap, 0, q.F, q.g_ux, q.g_uy, q.g_uzz, q.overlaps, nullptr, job->ws,
                               ws_bytes, sl.stream);
  if (rc != TNRG_OK) return rc;
  const size_t nt = (size_t)q.K * q.R;
  if (sl.flags_cap < nt) {
    if (sl.host_flags) (void)hipHostFree(sl.host_flags);
    sl.host_flags = nullptr;
    sl.flags_cap = 0;
    if (hipHostMalloc((void**)&sl.host_flags, nt * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return err(TNRG_EHIP, "hipHostMalloc of %zu flags failed", nt);
    sl.flags_cap = nt;
  }
  // the flags sit at offset 0 of the workspace
  hipError_t e = hipMemcpyAsync(sl.host_flags, job->ws, nt * sizeof(int32_t), hipMemcpyDeviceToHost,
                                sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) return err(TNRG_EHIP, "flag copy / event: %s", hipGetErrorString(e));
  return TNRG_OK;
}

// Collect finished launches.
int reap(tnrg_server* s) {
  for (size_t si = 0; si < s->slots.size(); ++si) {
    Slot& sl = s->slots[si];
    if (!sl.job) continue;
    hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    std::unique_ptr<Job> job = std::move(sl.job);
    s->arena.release(job->ws);
    job->ws = nullptr;
    if (e != hipSuccess) {
      complete(s, std::move(job), err(TNRG_EHIP, "request failed: %s", hipGetErrorString(e)));
      continue;
    }
    int any = 0;
    const size_t nt = (size_t)job->req.K * job->req.R;
    for (size_t t = 0; t < nt; ++t) any |= sl.host_flags[t];
    if ((any & TNRG_FLAG_OVERFLOW) && job->req.dcap == 0 && job->bucket + 1 < job->buckets.size()) {
      job->bucket += 1;  // regrow and retry before anything else
      s->regrown += 1;
      s->queue.push_front(std::move(job));
      continue;
    }
    int status = TNRG_OK;
    const tnrg_model& jm = job->model;
    int cap_max = jm.chi;
    if (jm.n / 2 < 30 && (1 << (jm.n / 2)) < cap_max) cap_max = 1 << (jm.n / 2);
    if ((any & TNRG_FLAG_OVERFLOW) && job->req.dcap == 0 && job->buckets[job->bucket] < cap_max)
      status = err(TNRG_EUNSUPPORTED, "request needs a capacity above the server's max_dcap %d",
                   s->max_dcap);
    else if (any & TNRG_FLAG_OVERFLOW)
      status = TNRG_EOVERFLOW;
    else if (any & TNRG_FLAG_NOCONV)
      status = TNRG_ENOCONV;
    else if (any & TNRG_FLAG_NONFINITE)
      status = TNRG_ENONFINITE;
    if (status == TNRG_OK && job->req.dcap == 0) {
      const tnrg_model& m = job->model;
      plan_put(PlanKey(m.n, m.m, m.chi, m.xt_model, job->req.K, job->req.R), job->buckets[job->bucket]);
    }
    complete(s, std::move(job), status);
  }
  return TNRG_OK;
}

// Admit queued requests in arrival order while slots and arena blocks allow.
void admit(tnrg_server* s) {
  size_t qi = 0;
  Job* blocked_head = nullptr;
  while (qi < s->queue.size()) {
    int free_slot = -1;
    for (size_t si = 0; si < s->slots.size(); ++si)
      if (!s->slots[si].job) {
        free_slot = (int)si;
        break;
      }
    if (free_slot < 0) return;
    Job* job = s->queue[qi].get();
    const int cap = job->buckets[job->bucket];
    const size_t need = grape_workspace_bytes(&job->model, job->req.K, job->req.R, cap, 0);
    if (need == 0 || need > s->arena.size()) {
      std::unique_ptr<Job> j = std::move(s->queue[qi]);
      s->queue.erase(s->queue.begin() + qi);
      complete(s, std::move(j),
               err(TNRG_ENOMEM, "request needs %zu workspace bytes, the arena holds %zu", need,
                   s->arena.size()));
      continue;
    }
    if (blocked_head && blocked_head->bypassed >= s->max_bypass) return;
    char* ws = s->arena.alloc(need);
    if (!ws) {
      if (!blocked_head) blocked_head = job;
      ++qi;
      continue;
    }
    if (blocked_head) blocked_head->bypassed += 1;
    job->ws = ws;
    job->launches += 1;
    if (!job->admitted_once) {
      job->admitted_once = true;
      job->t_admit = Clock::now();
      s->admitted += 1;
    }
    const int rc = launch(s, free_slot, job, need);
    std::unique_ptr<Job> j = std::move(s->queue[qi]);
    s->queue.erase(s->queue.begin() + qi);
    if (rc != TNRG_OK) {
      s->arena.release(ws);
      j->ws = nullptr;
      complete(s, std::move(j), rc);
      continue;
    }
    s->slots[free_slot].job = std::move(j);
  }
}

}  // namespace

extern "C" {

int tnrg_server_create(void* arena, size_t arena_bytes, int32_t n_streams, int32_t max_bypass,
                       int32_t max_dcap, tnrg_server** out) {
  if (!out) return err(TNRG_EINVAL, "NULL output pointer");
  *out = nullptr;
  if (!arena || arena_bytes < 256) return err(TNRG_EINVAL, "arena must be a device block of >= 256 bytes");
  if (n_streams < 1 || n_streams > 16) return err(TNRG_EINVAL, "n_streams = %d outside [1, 16]", n_streams);
  if (max_bypass < 0) return err(TNRG_EINVAL, "max_bypass < 0");
  if (max_dcap < 0) return err(TNRG_EINVAL, "max_dcap < 0");
  std::unique_ptr<tnrg_server> s(new (std::nothrow) tnrg_server(static_cast<char*>(arena), arena_bytes));
  if (!s) return err(TNRG_ENOMEM, "host allocation failed");
  s->max_bypass = max_bypass;
  s->max_dcap = max_dcap > 0 ? max_dcap : 1 << 30;
  s->slots.resize(n_streams);
  for (auto& sl : s->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      tnrg_server_destroy(s.release());
      return err(TNRG_EHIP, "stream/event creation: %s", hipGetErrorString(e));
    }
  }
  *out = s.release();
  return TNRG_OK;
}

int tnrg_server_submit(tnrg_server* s, const tnrg_request* req, int64_t* ticket) {
  if (!s || !req || !ticket) return err(TNRG_EINVAL, "NULL server, request or ticket");
  const tnrg_model* md = req->md;
  if (!md || !req->inputs || !req->targets) return err(TNRG_EINVAL, "NULL model or batches");
  if (md->n < 2 || md->m < 1 || !md->zz_mask || !md->xt_mask)
    return err(TNRG_EINVAL, "bad model (n = %d, m = %d)", md->n, md->m);
  if (req->K < 1 || req->R < 1 || req->dcap < 0) return err(TNRG_EINVAL, "bad K, R or dcap");
  if (!req->ux || !req->uy || !req->uzz || !req->J || !req->F || !req->g_ux || !req->g_uy ||
      !req->g_uzz)
    return err(TNRG_EINVAL, "NULL control, crosstalk or output buffer");
  std::unique_ptr<Job> job(new (std::nothrow) Job);
  if (!job) return err(TNRG_ENOMEM, "host allocation failed");
  job->req = *req;
  job->model = *md;
  job->zz.assign(md->zz_mask, md->zz_mask + (md->n - 1));
  job->xt.assign(md->xt_mask, md->xt_mask + (md->n - 1));
  job->model.zz_mask = job->zz.data();
  job->model.xt_mask = job->xt.data();
  job->req.md = &job->model;
  job->in = *req->inputs;
  job->tg = *req->targets;
  job->req.inputs = &job->in;
  job->req.targets = &job->tg;
  if (req->dcap > s->max_dcap)
    return err(TNRG_EUNSUPPORTED, "dcap %d above the server's max_dcap %d", req->dcap, s->max_dcap);
  if (req->dcap > 0) {
    job->buckets = {req->dcap};
  } else {
    job->buckets = bucket_sequence(job->model, plan_get(PlanKey(md->n, md->m, md->chi, md->xt_model, req->K, req->R)),
                                   s->max_dcap, std::max(job->in.dcap, job->tg.dcap));
  }
  job->ticket = s->next_ticket++;
  job->t_submit = Clock::now();
  *ticket = job->ticket;
  s->queue.push_back(std::move(job));
  s->submitted += 1;
  return TNRG_OK;
}

int tnrg_server_progress(tnrg_server* s, tnrg_completion* done, int32_t max_done, int32_t* n_done) {
  if (!s || !n_done || max_done < 0 || (max_done > 0 && !done))
    return err(TNRG_EINVAL, "bad progress arguments");
  reap(s);
  admit(s);
  int n = 0;
  while (n < max_done && !s->finished.empty()) {
    done[n++] = s->finished.front();
    s->finished.pop_front();
  }
  *n_done = n;
  return TNRG_OK;
}

int tnrg_server_cancel_queued(tnrg_server* s, int64_t* tickets, int32_t max, int32_t* n) {
  if (!s || !n || max < 0 || (max > 0 && !tickets)) return err(TNRG_EINVAL, "bad cancel arguments");
  int k = 0;
  for (auto& j : s->queue) {
    if (k < max) tickets[k] = j->ticket;
    ++k;
  }
  s->cancelled += (int64_t)s->queue.size();
  s->queue.clear();
  *n = k < max ? k : max;
  return TNRG_OK;
}

int tnrg_server_info_get(const tnrg_server* s, tnrg_server_info* info) {
  if (!s || !info) return err(TNRG_EINVAL, "NULL server or info");
  memset(info, 0, sizeof *info);
  info->queued = (int32_t)s->queue.size();
  for (auto& sl : s->slots) info->running += sl.job ? 1 : 0;
  info->submitted = s->submitted;
  info->admitted = s->admitted;
  info->completed = s->completed;
  info->regrown = s->regrown;
  info->cancelled = s->cancelled;
  info->arena_bytes = s->arena.size();
  info->arena_free = s->arena.free_bytes();
  info->arena_largest_free = s->arena.largest_free();
  return TNRG_OK;
}

int tnrg_server_destroy(tnrg_server* s) {
  if (!s) return TNRG_OK;
  int rc = TNRG_OK;
  for (auto& sl : s->slots) {
    if (sl.stream && hipStreamSynchronize(sl.stream) != hipSuccess) rc = TNRG_EHIP;
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.host_flags) (void)hipHostFree(sl.host_flags);
  }
  delete s;
  return rc == TNRG_OK ? TNRG_OK : err(rc, "a running request failed during shutdown");
}

}  // extern "C"
