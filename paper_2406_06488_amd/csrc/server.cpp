// Continuous-batching server.
//
// Requests arrive from any thread.  A scheduler thread owns one HIP stream and
// a fixed table of resident slots.  Each scheduler step:
//   1. admits queued requests in arrival order while a slot is free and the
//      device bytes held plus the request's footprint fit the memory budget;
//   2. runs the block stage (staging, Gram + epilogue, sums, centring) and the
//      split stream for the newly admitted requests -- their blocks then stay
//      resident in HBM;
//   3. gives every resident request its next range of split-column chunks of
//      the resampling stage, sized so that the whole step stays near
//      `chunk_updates` block-entry x split updates; all of it goes out as one
//      batched launch per kernel;
//   4. finishes the requests whose last chunk ran (statistics, count,
//      p-value), copies their results back and releases their memory.
// A request's numbers do not depend on what shares its steps: its reduction
// order is fixed by its own plan, and chunks only select split columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace et;

namespace {

// Best-fit arena over one device allocation made when the server starts.  Requests are
// placed and released on the host; a region is released only after the step that
// finished its request has synchronised, so it can be handed out again at once.
class Arena {
 public:
  bool init(size_t bytes) {
    bytes &= ~size_t(255);
    if (bytes == 0 || hipMalloc(&base_, bytes) != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      return false;
    }
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  void destroy() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
    free_.clear();
  }
  void* alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return nullptr;
    const size_t off = best->first, rem = best->second - n;
    free_.erase(best);
    if (rem) free_[off + n] = rem;
    return base_ + off;
  }
  bool owns(const void* p) const {
    return base_ && (const char*)p >= base_ && (const char*)p < base_ + size_;
  }
  void release(void* p, size_t n) {
    n = (n + 255) & ~size_t(255);
    size_t off = (size_t)((char*)p - base_);
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

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

struct Req {
  uint64_t id = 0;
  etest_request r{};
  TestPlan plan;
  int64_t footprint = 0;
  int slot = -1;
  void* ws = nullptr;
  int pc_total = 0, pc_done = 0;
  bool front_pending = true;
  bool done = false;
  etest_status status = ETEST_EBUSY;
  std::string err;
  etest_result result{};
};

}  // namespace

struct etest_server {
  etest_server_config cfg{};
  int device = 0;
  hipStream_t st = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::deque<Req*> pending;
  std::vector<Req*> slots;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  int64_t bytes_held = 0, completed = 0;
  // scheduler time per phase (seconds) and step count, printed at destroy when the
  // environment variable ETEST_SERVER_STATS is set
  double t_admit = 0, t_prep = 0, t_sync = 0, t_finish = 0;
  int64_t steps = 0;
  Arena arena;  // request workspaces; the stream-ordered pool serves what does not fit
  // device tables over the slot index space
  TestDesc* d_descs = nullptr;
  int64_t* d_offs = nullptr;   // [S_COUNT + 2][R + 1]: launch slots, then front / finish selectors
  int32_t* d_pcr = nullptr;    // [R][2]
  DevResult* d_results = nullptr;
  // pinned staging
  TestDesc* h_descs = nullptr;
  int64_t* h_offs = nullptr;
  int32_t* h_pcr = nullptr;
  DevResult* h_results = nullptr;
};

namespace {

constexpr int SEL_FRONT = S_COUNT, SEL_FINISH = S_COUNT + 1, NSEL = S_COUNT + 2;

etest_status serr(etest_status s, const char* m) { return set_error(s, m); }

void run_scheduler(etest_server* S);

}  // namespace

extern "C" etest_status etest_server_create(const etest_server_config* cfg, etest_server** out) {
  if (!cfg || !out) return serr(ETEST_EINVAL, "NULL argument");
  if (cfg->memory_budget_bytes <= 0 || cfg->max_resident < 1 || cfg->max_queue < 1)
    return serr(ETEST_EINVAL, "budget, max_resident and max_queue must be positive");
  init_pool_once();
  etest_server* S = new etest_server();
  S->cfg = *cfg;
  if (S->cfg.chunk_updates <= 0) S->cfg.chunk_updates = (int64_t)5e11;
  const int R = cfg->max_resident;
  S->slots.assign((size_t)R, nullptr);
  hipError_t e = hipGetDevice(&S->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&S->d_descs, sizeof(TestDesc) * R);
  if (e == hipSuccess) e = hipMalloc((void**)&S->d_offs, sizeof(int64_t) * NSEL * (R + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&S->d_pcr, sizeof(int32_t) * 2 * R);
  if (e == hipSuccess) e = hipMalloc((void**)&S->d_results, sizeof(DevResult) * R);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_descs, sizeof(TestDesc) * R, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_offs, sizeof(int64_t) * NSEL * (R + 1), 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_pcr, sizeof(int32_t) * 2 * R, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_results, sizeof(DevResult) * R, 0);
  if (e != hipSuccess) {
    set_error(ETEST_EDEVICE, std::string("server setup: ") + hipGetErrorString(e));
    etest_server_destroy(S);
    return ETEST_EDEVICE;
  }
  memset(S->h_descs, 0, sizeof(TestDesc) * R);
  // one allocation for the budget (smaller if the device cannot hold it all)
  for (size_t b = (size_t)cfg->memory_budget_bytes; b >= ((size_t)1 << 26); b /= 2)
    if (S->arena.init(b)) break;
  S->th = std::thread(run_scheduler, S);
  *out = S;
  return ETEST_OK;
}

extern "C" etest_status etest_server_submit(etest_server* S, const etest_request* req,
                                            uint64_t* id) {
  if (!S || !req || !id) return serr(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_request(*req);
  if (s != ETEST_OK) return s;
  Req* q = new Req();
  q->r = *req;
  q->plan = make_plan(*req);
  s = check_launch_sizes(&q->plan, 1);
  if (s != ETEST_OK) {
    delete q;
    return s;
  }
  q->footprint = (int64_t)q->plan.bytes;
  q->pc_total = (int)(q->plan.d.B_pad / NP);
  if (q->footprint > S->cfg.memory_budget_bytes) {
    delete q;
    return serr(ETEST_ENOMEM, "request footprint exceeds the server memory budget");
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if ((int64_t)S->pending.size() >= S->cfg.max_queue) {
      delete q;
      return serr(ETEST_EBUSY, "server queue is full");
    }
    q->id = S->next_id++;
    S->reqs[q->id] = q;
    S->pending.push_back(q);
    *id = q->id;
  }
  S->cv_work.notify_one();
  return ETEST_OK;
}

static etest_status take_result(etest_server* S, uint64_t id, etest_result* out, bool block) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return serr(ETEST_ENOTFOUND, "unknown request id");
  Req* q = it->second;
  if (block) S->cv_done.wait(lk, [&] { return q->done; });
  if (!q->done) return serr(ETEST_EBUSY, "request still running");
  etest_status s = q->status;
  if (s == ETEST_OK) *out = q->result;
  else set_error(s, q->err);
  S->reqs.erase(it);
  delete q;
  return s;
}

extern "C" etest_status etest_server_poll(etest_server* S, uint64_t id, etest_result* out) {
  if (!S || !out) return serr(ETEST_EINVAL, "NULL argument");
  return take_result(S, id, out, false);
}

extern "C" etest_status etest_server_wait(etest_server* S, uint64_t id, etest_result* out) {
  if (!S || !out) return serr(ETEST_EINVAL, "NULL argument");
  return take_result(S, id, out, true);
}

extern "C" etest_status etest_server_stats(etest_server* S, int64_t* queued, int64_t* resident,
                                           int64_t* bytes_held, int64_t* completed) {
  if (!S) return serr(ETEST_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t res = 0;
  for (Req* q : S->slots) res += q ? 1 : 0;
  if (queued) *queued = (int64_t)S->pending.size();
  if (resident) *resident = res;
  if (bytes_held) *bytes_held = S->bytes_held;
  if (completed) *completed = S->completed;
  return ETEST_OK;
}

extern "C" etest_status etest_server_destroy(etest_server* S) {
  if (!S) return serr(ETEST_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto& kv : S->reqs) delete kv.second;
  if (getenv("ETEST_SERVER_STATS"))
    fprintf(stderr,
            "etest server: %lld steps, %lld completed; scheduler seconds: admit %.3f, "
            "prepare+enqueue %.3f, device wait %.3f, finish %.3f\n",
            (long long)S->steps, (long long)S->completed, S->t_admit, S->t_prep, S->t_sync,
            S->t_finish);
  if (S->st) (void)hipStreamSynchronize(S->st);
  if (S->d_descs) (void)hipFree(S->d_descs);
  if (S->d_offs) (void)hipFree(S->d_offs);
  if (S->d_pcr) (void)hipFree(S->d_pcr);
  if (S->d_results) (void)hipFree(S->d_results);
  if (S->h_descs) (void)hipHostFree(S->h_descs);
  if (S->h_offs) (void)hipHostFree(S->h_offs);
  if (S->h_pcr) (void)hipHostFree(S->h_pcr);
  if (S->h_results) (void)hipHostFree(S->h_results);
  if (S->st) (void)hipStreamDestroy(S->st);
  S->arena.destroy();
  delete S;
  return ETEST_OK;
}

namespace {

// Block-entry x split updates of one split-column chunk of a request.
double chunk_cost(const Req* q) {
  return (double)q->plan.d.ntiles * TILE * TILE * NP;
}

void release_ws(etest_server* S, Req* q) {
  if (S->arena.owns(q->ws)) S->arena.release(q->ws, (size_t)q->footprint);
  else (void)hipFreeAsync(q->ws, S->st);
  q->ws = nullptr;
}

void fail_request(etest_server* S, Req* q, etest_status s, const std::string& m) {
  q->status = s;
  q->err = m;
  q->done = true;
  S->completed++;
}

void run_scheduler(etest_server* S) {
  (void)hipSetDevice(S->device);
  const int R = S->cfg.max_resident;
  std::vector<int> fresh, finishing;
  using clk = std::chrono::steady_clock;
  auto secs = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  while (true) {
    fresh.clear();
    finishing.clear();
    clk::time_point ta;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto any_resident = [&] {
        for (Req* q : S->slots)
          if (q) return true;
        return false;
      };
      S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || any_resident(); });
      if (S->stop && !any_resident() && S->pending.empty()) break;
      if (S->stop) {
        // fail whatever never got admitted
        while (!S->pending.empty()) {
          Req* q = S->pending.front();
          S->pending.pop_front();
          fail_request(S, q, ETEST_EDEVICE, "server shut down before the request ran");
        }
        S->cv_done.notify_all();
      }
      // 1. admission in arrival order
      ta = clk::now();
      while (!S->pending.empty()) {
        Req* q = S->pending.front();
        int slot = -1;
        for (int k = 0; k < R; ++k)
          if (!S->slots[(size_t)k]) {
            slot = k;
            break;
          }
        if (slot < 0 || S->bytes_held + q->footprint > S->cfg.memory_budget_bytes) break;
        S->pending.pop_front();
        void* ws = S->arena.alloc((size_t)q->footprint);
        hipError_t e = hipSuccess;
        if (!ws) e = hipMallocAsync(&ws, (size_t)q->footprint, S->st);
        if (e != hipSuccess || !ws) {
          (void)hipGetLastError();
          if (S->bytes_held == 0) {
            fail_request(S, q, ETEST_ENOMEM, "device memory exhausted");
            S->cv_done.notify_all();
            continue;
          }
          S->pending.push_front(q);  // retry once others release memory
          break;
        }
        q->ws = ws;
        q->slot = slot;
        assign_pointers(q->plan, (char*)ws, S->d_results + slot);
        S->slots[(size_t)slot] = q;
        S->bytes_held += q->footprint;
        fresh.push_back(slot);
      }
    }
    const clk::time_point tb = clk::now();
    // 2-4. one step of device work over the slot table
    int64_t* O = S->h_offs;
    memset(O, 0, sizeof(int64_t) * NSEL * (R + 1));
    for (int k = 0; k < R; ++k) S->h_pcr[2 * k] = S->h_pcr[2 * k + 1] = 0;
    int nres = 0;
    for (int k = 0; k < R; ++k) nres += S->slots[(size_t)k] ? 1 : 0;
    const double share = nres > 0 ? (double)S->cfg.chunk_updates / nres : 0.0;
    // the split streams of this step's fresh requests: 32 splits per workgroup once they
    // outgrow the chip, as in build_batch (the split words are the same either way)
    int64_t member_wg = 0;
    for (int k = 0; k < R; ++k) {
      const Req* q = S->slots[(size_t)k];
      if (q && q->front_pending) member_wg += q->plan.wg[S_MEMBER];
    }
    const bool member_wide = member_wg > MEMBER_WIDE_MIN_WG;
    bool any = false;
    for (int k = 0; k < R; ++k) {
      Req* q = S->slots[(size_t)k];
      int64_t w[NSEL] = {};
      if (q) {
        const TestPlan& P = q->plan;
        if (q->front_pending) {
          for (int s : {S_COLPART, S_COLMEAN, S_STAGE, S_MEMBER, S_ROWSUM, S_CENTER_F64,
                        S_CENTER_SPLIT})
            w[s] = P.wg[s];
          for (int s : GRAM_SLOTS) w[s] = P.wg[s];
          if (member_wide && P.wg[S_MEMBER] > 0) w[S_MEMBER] = P.d.B_pad / MEMBER_SPLITS_WIDE;
          w[SEL_FRONT] = 1;
        }
        const int left = q->pc_total - q->pc_done;
        int take = (int)std::max(1.0, share / chunk_cost(q));
        take = std::min(take, left);
        S->h_pcr[2 * k] = q->pc_done;
        S->h_pcr[2 * k + 1] = take;
        const int64_t units = perm_units(P.d, take);
        for (int s : {S_PERM_F64, S_PERM_S2, S_PERM_S3})
          if (P.wg[s] > 0) w[s] = units;
        q->pc_done += take;
        if (q->pc_done == q->pc_total) {
          w[S_PSTAT] = P.wg[S_PSTAT];
          w[SEL_FINISH] = 1;
          finishing.push_back(k);
        }
        any = true;
      }
      for (int s = 0; s < NSEL; ++s) O[(size_t)s * (R + 1) + k + 1] = O[(size_t)s * (R + 1) + k] + w[s];
    }
    if (!any) continue;
    for (int k : fresh) S->h_descs[k] = S->slots[(size_t)k]->plan.d;
    hipError_t e = hipSuccess;
    for (int k : fresh)
      if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_descs + k, S->h_descs + k, sizeof(TestDesc), hipMemcpyHostToDevice,
                           S->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->d_offs, O, sizeof(int64_t) * NSEL * (R + 1), hipMemcpyHostToDevice, S->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->d_pcr, S->h_pcr, sizeof(int32_t) * 2 * R, hipMemcpyHostToDevice, S->st);
    auto offs = [&](int s) { return S->d_offs + (size_t)s * (R + 1); };
    auto total = [&](int s) { return O[(size_t)s * (R + 1) + R]; };
    const TestDesc* D = S->d_descs;
    hipStream_t st = S->st;
    if (e == hipSuccess) {
      if (total(SEL_FRONT) > 0) {
        launch_clear_flags(st, D, offs(SEL_FRONT), R);
        launch_colpart(total(S_COLPART), st, D, offs(S_COLPART), R);
        launch_colmean(total(S_COLMEAN), st, D, offs(S_COLMEAN), R);
        launch_stage(total(S_STAGE), st, D, offs(S_STAGE), R);
        launch_gram_slots(offs, total, st, D, R, false);
        launch_member(total(S_MEMBER), st, D, offs(S_MEMBER), R, member_wide);
        launch_rowsum(total(S_ROWSUM), st, D, offs(S_ROWSUM), R);
        launch_observed(st, D, offs(SEL_FRONT), R);
        launch_center(true, total(S_CENTER_F64), st, D, offs(S_CENTER_F64), R);
        launch_center(false, total(S_CENTER_SPLIT), st, D, offs(S_CENTER_SPLIT), R);
      }
      launch_perm(0, total(S_PERM_F64), st, D, offs(S_PERM_F64), R, S->d_pcr);
      launch_perm(2, total(S_PERM_S2), st, D, offs(S_PERM_S2), R, S->d_pcr);
      launch_perm(3, total(S_PERM_S3), st, D, offs(S_PERM_S3), R, S->d_pcr);
      if (total(SEL_FINISH) > 0) {
        launch_pstat(total(S_PSTAT), st, D, offs(S_PSTAT), R);
        e = hipMemcpyAsync(S->h_results, S->d_results, sizeof(DevResult) * R,
                           hipMemcpyDeviceToHost, st);
      }
      if (e == hipSuccess) e = hipGetLastError();
    }
    const clk::time_point tc = clk::now();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const clk::time_point td = clk::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (int k : fresh)
        if (S->slots[(size_t)k]) S->slots[(size_t)k]->front_pending = false;
      if (e != hipSuccess) {
        // a device error ends every resident request
        for (int k = 0; k < R; ++k) {
          Req* q = S->slots[(size_t)k];
          if (!q) continue;
          fail_request(S, q, ETEST_EDEVICE, std::string("device: ") + hipGetErrorString(e));
          release_ws(S, q);
          S->bytes_held -= q->footprint;
          S->slots[(size_t)k] = nullptr;
        }
      } else {
        for (int k : finishing) {
          Req* q = S->slots[(size_t)k];
          etest_result tmp{};
          etest_status s = dev_to_result(S->h_results[k], &tmp);
          q->status = s;
          if (s == ETEST_OK) q->result = tmp;
          else q->err = etest_last_error();
          q->done = true;
          S->completed++;
          release_ws(S, q);
          S->bytes_held -= q->footprint;
          S->slots[(size_t)k] = nullptr;
        }
      }
      S->t_admit += secs(ta, tb);
      S->t_prep += secs(tb, tc);
      S->t_sync += secs(tc, td);
      S->t_finish += secs(td, clk::now());
      S->steps++;
    }
    S->cv_done.notify_all();
  }
}

}  // namespace
