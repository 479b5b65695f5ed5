// Request server: continuous admission of GLCM jobs of mixed image size, N
// and offset lists onto lanes (HIP streams), bounded by an HBM budget.
//
// One scheduler thread admits queued requests in arrival order.  A request
// is admitted as soon as a lane is idle and its device memory fits: its
// server-owned results (first fit in a device pool) plus, if the lane has no
// plan for its (dtype, N) yet, that plan's workspace; idle plans are evicted,
// least recently used first, to make room.  The lane's plan is re-targeted at
// the request's offsets (glcm_plan_rebind: no allocation), the counts and
// statistics are queued on the lane's stream, and a host function queued
// behind them hands the lane back the moment they complete, which wakes the
// scheduler for the next request.  Requests on different lanes overlap on the
// GPU; results stay in device memory until fetched or released.
//
// Host images: a request may bring its image in host memory (pinned or
// pageable); the lane's plan streams it to the GPU in row tiles (glcm_compute's
// host path: a pageable image is first copied into pinned staging by the
// scheduler thread), and the tile buffers the plan allocates count against the
// budget from then on.
//
// Continuous batching: when the admitted request is small (at most
// kFusePixels pixels, at most four offsets of reach <= 2), queued requests of
// the same job (dtype, N, range, offsets, statistics or not) that are small
// too join it, in arrival order, as far as their results fit: the group runs
// as one persistent batch launch (the fused batch kernel of glcm_batch_compute,
// each image's counts and statistics written straight to its request's
// buffers) and completes together.
//
// Locking: one mutex guards the server state.  No HIP call is made while it
// is held (hipMalloc / hipFree may wait for queued work, whose completion
// callbacks take the mutex).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "glcm.h"
#include "glcm_host.h"

namespace {

constexpr int kMaxLanes = 16;
constexpr uint64_t kAlign = 256;
// plans are created for at least this many offsets (the 12 of d in {1, 2, 4}
// at four angles) and re-targeted per request
constexpr int kPlanMinK = 12;
constexpr int kPlanMaxSide = 65535;
constexpr uint64_t kXbufCap = 256ull << 20;  // plans keep per-XCD accumulators up to this size
// continuous batching: requests of at most kFusePixels pixels, groups of at
// most kFuseMax requests, companions looked for among the first kFuseScan
// queued requests
constexpr uint64_t kFusePixels = 1ull << 20;
constexpr int kFuseMax = 1024;
constexpr int kFuseScan = 4096;

using Clock = std::chrono::steady_clock;

uint64_t round_up(uint64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over byte offsets [0, size) of the result pool.
class Pool {
 public:
  void init(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t start = it->first + bytes, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
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

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length of each free run
};

struct Request;

struct LanePlan {
  glcm_plan_t plan = nullptr;
  int dtype = 0, N = 0, kcap = 0;
  uint64_t bytes = 0;     // budgeted workspace
  uint64_t last_use = 0;  // admission counter value of its last request
};

struct Lane {
  hipStream_t stream = nullptr;
  std::vector<LanePlan> plans;
  Request* cur = nullptr;  // running request, null when idle
};

struct Request {
  glcm_server_s* srv = nullptr;
  uint64_t id = 0;
  glcm_request_t r{};
  glcm_offset_t offs[GLCM_MAX_OFFSETS];
  uint64_t res_bytes = 0, res_off = 0;  // pool bytes held for server-owned results
  uint64_t out_bytes = 0;
  uint32_t* out = nullptr;
  float* feat = nullptr;
  int lane = -1;
  bool done = false;
  int status = GLCM_OK;
  int fused = 1;                  // requests in the launch that carried it
  bool host = false;              // image in host memory (streamed in row tiles; never fused)
  std::vector<Request*> group;    // the head of a fused launch: its other requests
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// A request the batch kernel can take in a fused launch: a small image, at
// most four offsets, each with |dx|, |dy| <= 2, levels in one byte.
bool fusable(const Request* q) {
  if (q->host || (uint64_t)q->r.W * (uint64_t)q->r.H > kFusePixels || q->r.K > 4 || q->r.N > 255) return false;
  for (int k = 0; k < q->r.K; ++k)
    if (std::abs(q->offs[k].dx) > 2 || std::abs(q->offs[k].dy) > 2) return false;
  return true;
}

// Same job: one plan binding and one quantizer serve both.
bool same_job(const Request* a, const Request* b) {
  return a->r.dtype == b->r.dtype && a->r.N == b->r.N && a->r.lo == b->r.lo && a->r.hi == b->r.hi &&
         a->r.K == b->r.K && (a->r.features != 0) == (b->r.features != 0) &&
         std::memcmp(a->offs, b->offs, sizeof(glcm_offset_t) * (size_t)a->r.K) == 0;
}

// Workspace a new plan for (N, kcap) reserves at creation: the per-XCD
// accumulators (16 slices of kcap * N * N words) when they fit the cap.
uint64_t plan_estimate(int N, int kcap) {
  const uint64_t x = 16ull * (uint64_t)kcap * (uint64_t)N * (uint64_t)N * 4ull;
  return x <= kXbufCap ? x : 0;
}

// What the scheduler decided for one admission (applied outside the lock).
struct Admission {
  Request* q = nullptr;
  int lane = -1;
  bool need_plan = false;
  int kcap = 0;
  std::vector<glcm_plan_t> evict;
};

}  // namespace

struct glcm_server_s {
  int device = 0;
  Clock::time_point t0;
  std::vector<Lane> lanes;
  uint64_t budget = 0, pool_bytes = 0;
  char* pool_base = nullptr;
  Pool pool;
  uint64_t held = 0, max_held = 0;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1, submitted = 0, completed = 0, failed = 0, admissions = 0;
  uint64_t fused_launches = 0, fused_requests = 0;
  int inflight = 0, max_inflight = 0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::thread sched;
  bool stop = false;

  double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

void note_held(glcm_server_s* s) { s->max_held = std::max(s->max_held, s->held); }

// Marks a request finished (lock held): the lane goes idle, waiters wake up.
void finish_locked(glcm_server_s* s, Request* q, int status) {
  q->status = status;
  q->done = true;
  q->t_done = s->now_us();
  if (q->lane >= 0 && s->lanes[q->lane].cur == q) s->lanes[q->lane].cur = nullptr;
  s->inflight--;
  if (status == GLCM_OK)
    s->completed++;
  else
    s->failed++;
  s->cv_sched.notify_all();
  s->cv_done.notify_all();
}

// Finishes a launch's head request and the requests fused with it (lock held).
void finish_group_locked(glcm_server_s* s, Request* q, int status) {
  for (Request* m : q->group) finish_locked(s, m, status);
  q->group.clear();
  finish_locked(s, q, status);
}

// Runs on the HIP runtime's callback thread once the request's work is done.
void on_done(void* arg) {
  Request* q = static_cast<Request*>(arg);
  glcm_server_s* s = q->srv;
  std::lock_guard<std::mutex> lk(s->mu);
  finish_group_locked(s, q, GLCM_OK);
}

// Points a request's missing result buffers into the pool block at `off`.
void place_results(glcm_server_s* s, Request* q, uint64_t off) {
  q->res_off = off;
  if (!q->r.out) q->out = reinterpret_cast<uint32_t*>(s->pool_base + off);
  if (q->r.features && !q->r.feat)
    q->feat = reinterpret_cast<float*>(s->pool_base + off + (q->r.out ? 0 : round_up(q->out_bytes)));
}

// Admits queued requests of the head's job into its launch (lock held): small
// ones, in arrival order, while their results fit the budget and the pool.
void gather_locked(glcm_server_s* s, Request* head) {
  if (!fusable(head)) return;
  const size_t scan = std::min(s->queue.size(), (size_t)kFuseScan);
  std::vector<char> taken(scan, 0);
  size_t ntaken = 0;
  for (size_t i = 0; i < scan && head->group.size() + 1 < (size_t)kFuseMax; ++i) {
    Request* r = s->queue[i];
    if (!same_job(head, r) || !fusable(r)) continue;
    if (s->held + r->res_bytes > s->budget) break;
    uint64_t off = 0;
    if (r->res_bytes && !s->pool.alloc(r->res_bytes, &off)) break;
    s->held += r->res_bytes;
    place_results(s, r, off);
    r->lane = head->lane;
    r->t_admit = head->t_admit;
    s->inflight++;
    head->group.push_back(r);
    taken[i] = 1;
    ++ntaken;
  }
  if (!ntaken) return;
  note_held(s);
  s->max_inflight = std::max(s->max_inflight, s->inflight);
  std::deque<Request*> rest;
  for (size_t i = 0; i < s->queue.size(); ++i)
    if (i >= scan || !taken[i]) rest.push_back(s->queue[i]);
  s->queue.swap(rest);
  const int n = (int)head->group.size() + 1;
  head->fused = n;
  for (Request* r : head->group) r->fused = n;
  s->fused_launches++;
  s->fused_requests += (uint64_t)n;
}

// Tries to admit the head of the queue (lock held).  Fills *a and returns
// true on success; leaves everything unchanged otherwise.
bool pick(glcm_server_s* s, Admission* a) {
  if (s->queue.empty()) return false;
  Request* q = s->queue.front();
  const int dtype = q->r.dtype, N = q->r.N, K = q->r.K;
  // an idle lane, preferring one that already has a plan this request fits
  int lane = -1, plan_idx = -1;
  for (int l = 0; l < (int)s->lanes.size(); ++l) {
    if (s->lanes[l].cur) continue;
    const auto& ps = s->lanes[l].plans;
    for (int i = 0; i < (int)ps.size(); ++i) {
      if (ps[i].dtype == dtype && ps[i].N == N && ps[i].kcap >= K) {
        lane = l;
        plan_idx = i;
        break;
      }
    }
    if (plan_idx >= 0) break;
    if (lane < 0) lane = l;
  }
  if (lane < 0) return false;
  Lane& L = s->lanes[lane];
  const bool need_plan = plan_idx < 0;
  const int kcap = std::max(K, kPlanMinK);
  const uint64_t plan_bytes = need_plan ? plan_estimate(N, kcap) : 0;
  // a smaller plan for the same (dtype, N) on this lane is replaced
  std::vector<std::pair<int, int>> victims;  // (lane, plan index)
  uint64_t freed = 0;
  if (need_plan) {
    for (int i = 0; i < (int)L.plans.size(); ++i)
      if (L.plans[i].dtype == dtype && L.plans[i].N == N) {
        victims.emplace_back(lane, i);
        freed += L.plans[i].bytes;
      }
  }
  // evict idle plans, least recently used first, until the request fits
  while (s->held - freed + plan_bytes + q->res_bytes > s->budget) {
    int bl = -1, bi = -1;
    uint64_t best = UINT64_MAX;
    for (int l = 0; l < (int)s->lanes.size(); ++l) {
      if (s->lanes[l].cur) continue;
      for (int i = 0; i < (int)s->lanes[l].plans.size(); ++i) {
        if (l == lane && i == plan_idx) continue;
        if (std::find(victims.begin(), victims.end(), std::make_pair(l, i)) != victims.end()) continue;
        if (s->lanes[l].plans[i].last_use < best) {
          best = s->lanes[l].plans[i].last_use;
          bl = l;
          bi = i;
        }
      }
    }
    if (bl < 0) return false;  // nothing idle left to evict: wait for a completion
    victims.emplace_back(bl, bi);
    freed += s->lanes[bl].plans[bi].bytes;
  }
  uint64_t off = 0;
  if (q->res_bytes && !s->pool.alloc(q->res_bytes, &off)) return false;  // wait for a release
  // commit
  s->queue.pop_front();
  std::sort(victims.begin(), victims.end(), [](auto x, auto y) { return x.second > y.second; });
  for (auto& v : victims) {
    auto& ps = s->lanes[v.first].plans;
    a->evict.push_back(ps[v.second].plan);
    ps.erase(ps.begin() + v.second);
  }
  s->held = s->held - freed + plan_bytes + q->res_bytes;
  note_held(s);
  place_results(s, q, off);
  q->lane = lane;
  q->t_admit = s->now_us();
  L.cur = q;
  s->inflight++;
  s->max_inflight = std::max(s->max_inflight, s->inflight);
  s->admissions++;
  gather_locked(s, q);
  if (!need_plan) L.plans[plan_idx].last_use = s->admissions;
  a->q = q;
  a->lane = lane;
  a->need_plan = need_plan;
  a->kcap = kcap;
  return true;
}

// Queues an admitted request's work on its lane (lock not held).
int launch(glcm_server_s* s, Admission& a) {
  for (glcm_plan_t p : a.evict) (void)glcm_plan_destroy(p);
  Request* q = a.q;
  Lane& L = s->lanes[a.lane];
  glcm_plan_t plan = nullptr;
  if (a.need_plan) {
    // created for kcap offsets (the request's, repeated) and re-targeted below
    glcm_offset_t capo[GLCM_MAX_OFFSETS];
    for (int k = 0; k < a.kcap; ++k) capo[k] = q->offs[k % q->r.K];
    int rc = glcm_plan_create(&plan, q->r.dtype, q->r.N, a.kcap, capo, kPlanMaxSide, kPlanMaxSide, 0);
    std::lock_guard<std::mutex> lk(s->mu);
    s->held -= plan_estimate(q->r.N, a.kcap);  // the estimate is replaced by what the plan holds
    if (rc != GLCM_OK) return rc;
    LanePlan lp;
    lp.plan = plan;
    lp.dtype = q->r.dtype;
    lp.N = q->r.N;
    lp.kcap = a.kcap;
    size_t wb = 0;
    (void)glcm_plan_workspace(plan, &wb);
    lp.bytes = wb;
    lp.last_use = s->admissions;
    s->held += wb;
    note_held(s);
    L.plans.push_back(lp);
  } else {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& lp : L.plans)
      if (lp.dtype == q->r.dtype && lp.N == q->r.N && lp.kcap >= q->r.K) {
        plan = lp.plan;
        break;
      }
  }
  if (!plan) return GLCM_EINVAL;
  int rc = glcm_plan_rebind(plan, q->offs, q->r.K);
  if (rc != GLCM_OK) return rc;
  // (the group is fixed once admitted: only this thread reads it until the
  // launch completes)
  if (!q->group.empty()) {
    // one fused batch launch for the whole group
    const size_t n = q->group.size() + 1;
    std::vector<glcm_tile_t> tiles(n);
    std::vector<uint32_t*> outs(n);
    std::vector<float*> feats(n);
    for (size_t i = 0; i < n; ++i) {
      const Request* m = i == 0 ? q : q->group[i - 1];
      tiles[i] = glcm_tile_t{m->r.img, m->r.stride, m->r.W, m->r.H};
      outs[i] = m->out;
      feats[i] = m->feat;
    }
    rc = glcm::batch_compute_to(plan, tiles.data(), (int)n, q->r.lo, q->r.hi, outs.data(),
                                q->r.features ? feats.data() : nullptr, L.stream);
    if (rc == GLCM_EUNSUPPORTED) {
      // a layout the batch kernel does not take (its LDS): one call each
      rc = GLCM_OK;
      for (size_t i = 0; i < n && rc == GLCM_OK; ++i) {
        const Request* m = i == 0 ? q : q->group[i - 1];
        rc = glcm_compute(plan, m->r.img, m->r.W, m->r.H, m->r.stride, m->r.dtype, m->r.N, m->r.lo, m->r.hi,
                          m->offs, m->r.K, m->out, L.stream);
        if (rc == GLCM_OK && m->r.features) rc = glcm_features(m->out, m->r.K, m->r.N, m->feat, L.stream);
      }
    }
  } else {
    rc = glcm_compute(plan, q->r.img, q->r.W, q->r.H, q->r.stride, q->r.dtype, q->r.N, q->r.lo, q->r.hi, q->offs,
                      q->r.K, q->out, L.stream);
    if (rc == GLCM_OK && q->r.features) rc = glcm_features(q->out, q->r.K, q->r.N, q->feat, L.stream);
  }
  {
    // band partials or tile buffers the call allocated count from now on
    size_t wb = 0;
    (void)glcm_plan_workspace(plan, &wb);
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& lp : L.plans)
      if (lp.plan == plan) {
        s->held = s->held - lp.bytes + wb;
        lp.bytes = wb;
        note_held(s);
      }
  }
  if (rc == GLCM_OK) {
    const hipError_t e = hipLaunchHostFunc(L.stream, on_done, q);
    if (e != hipSuccess) rc = glcm::hip_error_status(e);
  }
  if (rc != GLCM_OK) (void)hipStreamSynchronize(L.stream);  // nothing of it may still run
  return rc;
}

void scheduler(glcm_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Admission a;
    while (!pick(s, &a)) {
      if (s->stop && s->queue.empty()) return;
      s->cv_sched.wait(lk);
    }
    lk.unlock();
    const int rc = launch(s, a);
    lk.lock();
    if (rc != GLCM_OK) finish_group_locked(s, a.q, rc);
  }
}

Request* find_locked(glcm_server_s* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  return it == s->reqs.end() ? nullptr : it->second.get();
}

void fill_info(const Request* q, glcm_request_info_t* info) {
  std::memset(info, 0, sizeof(*info));
  info->done = q->done ? 1 : 0;
  info->status = q->status;
  info->lane = q->lane;
  info->fused = q->fused;
  info->submit_us = q->t_submit;
  info->admit_us = q->t_admit;
  info->done_us = q->t_done;
  info->out = q->out;
  info->feat = q->feat;
}

}  // namespace

extern "C" {

GLCM_API int glcm_server_create(glcm_server_t* srv, int lanes, uint64_t hbm_budget, uint64_t result_pool_bytes,
                                uint32_t flags) {
  if (!srv) return GLCM_EINVAL;
  *srv = nullptr;
  if (lanes < 1 || lanes > kMaxLanes || hbm_budget == 0 || result_pool_bytes > hbm_budget || flags != 0)
    return GLCM_EINVAL;
  std::unique_ptr<glcm_server_s> s(new (std::nothrow) glcm_server_s());
  if (!s) return GLCM_ENOMEM;
  s->t0 = Clock::now();
  s->budget = hbm_budget;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return glcm::hip_error_status(e);
  s->lanes.resize(lanes);
  for (auto& L : s->lanes) {
    e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (auto& M : s->lanes)
        if (M.stream) (void)hipStreamDestroy(M.stream);
      return glcm::hip_error_status(e);
    }
  }
  s->pool_bytes = result_pool_bytes / kAlign * kAlign;
  if (s->pool_bytes) {
    e = hipMalloc((void**)&s->pool_base, s->pool_bytes);
    if (e != hipSuccess) {
      for (auto& M : s->lanes) (void)hipStreamDestroy(M.stream);
      return glcm::hip_error_status(e);
    }
  }
  s->pool.init(s->pool_bytes);
  glcm_server_s* raw = s.get();
  try {
    s->sched = std::thread(scheduler, raw);
  } catch (...) {
    if (s->pool_base) (void)hipFree(s->pool_base);
    for (auto& M : s->lanes) (void)hipStreamDestroy(M.stream);
    return GLCM_ENOMEM;
  }
  *srv = s.release();
  return GLCM_OK;
}

GLCM_API int glcm_server_submit(glcm_server_t s, const glcm_request_t* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return GLCM_EINVAL;
  const glcm_request_t& r = *req;
  int rc = glcm::check_request_args(r.img, r.W, r.H, r.stride, r.dtype, r.N, r.lo, r.hi, r.offsets, r.K);
  if (rc != GLCM_OK) return rc;
  if (r.W > kPlanMaxSide || r.H > kPlanMaxSide) return GLCM_EINVAL;
  int dev = -1;
  const int img_kind = glcm::memory_kind(r.img, &dev);
  if (img_kind == 2 && dev != s->device) return GLCM_EINVAL;
  if (r.out && (glcm::memory_kind(r.out, &dev) != 2 || dev != s->device)) return GLCM_EINVAL;
  if (r.features && r.feat && (glcm::memory_kind(r.feat, &dev) != 2 || dev != s->device)) return GLCM_EINVAL;
  const uint64_t out_bytes = (uint64_t)r.K * (uint64_t)r.N * (uint64_t)r.N * 4ull;
  const uint64_t res = (r.out ? 0 : round_up(out_bytes)) + (r.features && !r.feat ? round_up((uint64_t)r.K * 20u) : 0);
  if (res && !s->pool_bytes) return GLCM_EINVAL;
  if (res > s->pool_bytes || res + plan_estimate(r.N, std::max(r.K, kPlanMinK)) > s->budget)
    return GLCM_EUNSUPPORTED;
  std::unique_ptr<Request> q(new (std::nothrow) Request());
  if (!q) return GLCM_ENOMEM;
  q->srv = s;
  q->r = r;
  std::memcpy(q->offs, r.offsets, sizeof(glcm_offset_t) * (size_t)r.K);
  q->r.offsets = q->offs;
  q->out_bytes = out_bytes;
  q->res_bytes = res;
  q->out = r.out;
  q->feat = r.features ? r.feat : nullptr;
  q->host = img_kind != 2;
  std::lock_guard<std::mutex> lk(s->mu);
  q->id = s->next_id++;
  q->t_submit = s->now_us();
  *ticket = q->id;
  s->queue.push_back(q.get());
  s->reqs.emplace(q->id, std::move(q));
  s->submitted++;
  s->cv_sched.notify_all();
  return GLCM_OK;
}

GLCM_API int glcm_server_query(glcm_server_t s, uint64_t ticket, glcm_request_info_t* info) {
  if (!s || !info) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const Request* q = find_locked(s, ticket);
  if (!q) return GLCM_EINVAL;
  fill_info(q, info);
  return GLCM_OK;
}

GLCM_API int glcm_server_wait(glcm_server_t s, uint64_t ticket, glcm_request_info_t* info) {
  if (!s) return GLCM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  // looked up again on every wake: another thread may release the ticket
  Request* q = nullptr;
  s->cv_done.wait(lk, [&] {
    q = find_locked(s, ticket);
    return !q || q->done;
  });
  if (!q) return GLCM_EINVAL;
  if (info) fill_info(q, info);
  return q->status;
}

GLCM_API int glcm_server_fetch(glcm_server_t s, uint64_t ticket, uint32_t* out, float* feat, void* stream) {
  if (!s || !out) return GLCM_EINVAL;
  const uint32_t* src = nullptr;
  const float* fsrc = nullptr;
  uint64_t bytes = 0, fbytes = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const Request* q = find_locked(s, ticket);
    if (!q || !q->done || q->status != GLCM_OK) return GLCM_EINVAL;
    src = q->out;
    fsrc = q->feat;
    bytes = q->out_bytes;
    fbytes = (uint64_t)q->r.K * 20u;
  }
  hipError_t e = hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e == hipSuccess && feat && fsrc) e = hipMemcpyAsync(feat, fsrc, fbytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return glcm::hip_error_status(e);
}

GLCM_API int glcm_server_release(glcm_server_t s, uint64_t ticket) {
  if (!s) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GLCM_EINVAL;
  Request* q = it->second.get();
  if (!q->done) return GLCM_EBUSY;
  if (q->res_bytes && q->lane >= 0) {  // admitted: its pool bytes were taken
    s->pool.release(q->res_off, q->res_bytes);
    s->held -= q->res_bytes;
  }
  s->reqs.erase(it);
  s->cv_sched.notify_all();
  return GLCM_OK;
}

GLCM_API int glcm_server_drain(glcm_server_t s) {
  if (!s) return GLCM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight == 0; });
  return GLCM_OK;
}

GLCM_API int glcm_server_stats(glcm_server_t s, glcm_server_stats_t* st) {
  if (!s || !st) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->lanes = (int32_t)s->lanes.size();
  st->max_inflight = s->max_inflight;
  st->budget_bytes = s->budget;
  st->bytes_in_use = s->held;
  st->max_bytes_in_use = s->max_held;
  st->fused_launches = s->fused_launches;
  st->fused_requests = s->fused_requests;
  return GLCM_OK;
}

GLCM_API int glcm_server_destroy(glcm_server_t s) {
  if (!s) return GLCM_OK;
  (void)glcm_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
  }
  if (s->sched.joinable()) s->sched.join();
  for (auto& L : s->lanes) {
    (void)hipStreamSynchronize(L.stream);
    for (auto& lp : L.plans) (void)glcm_plan_destroy(lp.plan);
    (void)hipStreamDestroy(L.stream);
  }
  if (s->pool_base) (void)hipFree(s->pool_base);
  delete s;
  return GLCM_OK;
}

}  // extern "C"
