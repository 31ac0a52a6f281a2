// Request server: many independent factorizations of mixed shapes in flight
// on one GPU (qrcp_server_* in qrcp.h).
//
// A fixed set of worker threads, each with its own HIP stream, takes requests
// from one FIFO queue as soon as they can be admitted, so requests that
// arrive while others run start as soon as a slot and device memory free up,
// and their kernels overlap on the device.  Device memory is one pool carved
// at creation (hbm_budget bytes): an admitted request gets a slice of it
// (first fit), returned when the request completes, so nothing is allocated
// or freed on the device while requests run.  Admission checks two budgets:
//   - device memory: the request's workspace fits a free slice of the pool;
//   - resident workgroups: the pivot-selection and sketch-QR-head kernels keep
//     all of their workgroups resident while they wait on each other, one
//     workgroup per compute unit (their LDS use); the running requests' largest
//     such grids must fit the device together, so two of them can never hold
//     compute units the other one is waiting for.
// Every request runs the same kernels as a lone qrcp_factor call on the same
// inputs, so its result is bitwise the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <map>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

struct qrcp_server {
  int device = 0;
  int slots = 4;
  int64_t budget = 0;
  int cu_budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  struct Job {
    qrcp_request req;
    qrcp_result res;
    int state = 0;  // 0 queued, 1 running, 2 done
    size_t ws = 0;
    int groups = 0;
  };
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Job> jobs;
  uint64_t next = 1;
  char* pool = nullptr;                 // device memory carved at creation
  std::map<size_t, size_t> free_list;   // offset -> bytes of the free slices
  int groups_used = 0;

  // first fit of `bytes` (256-byte multiples), or SIZE_MAX
  size_t take(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_list.erase(it);
      if (len > bytes) free_list[off + bytes] = len - bytes;
      return off;
    }
    return SIZE_MAX;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    auto it = free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace qrcp {
namespace {

int request_groups(const qrcp_request& r) {
  const int d = (int)std::ceil(r.sketch_factor * (double)r.block_size - 1e-12);
  const int bf = blockfact_groups((int)std::min<int64_t>(r.block_size, r.n));
  return std::max(std::max(lu_resident_groups(r.n), sketch_head_groups(d, r.n)), bf);
}

void worker_main(qrcp_server* s, int w) {
  (void)w;
  hipSetDevice(s->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  for (;;) {
    qrcp_server::Job* job = nullptr;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->queue.empty()) {
          if (s->stop) break;
          s->cv_work.wait(lk);
          continue;
        }
        qrcp_server::Job& j = s->jobs[s->queue.front()];
        if (s->groups_used + j.groups <= s->cu_budget) {
          off = s->take(j.ws);
          if (off != SIZE_MAX) {
            s->queue.pop_front();
            job = &j;
            job->state = 1;
            job->res.start_ms = s->now_ms();
            s->groups_used += j.groups;
            break;
          }
        }
        s->cv_work.wait(lk);
      }
    }
    if (!job) break;
    int rc = QRCP_OK;
    int64_t rank = 0;
    if (!st) rc = QRCP_ERR_HIP;
    if (rc == QRCP_OK) {
      const qrcp_request& r = job->req;
      rc = factor_served(r.A, r.m, r.n, r.lda, r.block_size, r.sketch_factor, r.seed, r.tol,
                         r.jpiv, r.tau, &rank, &r.opts, s->pool + off, job->ws, st);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      job->res.status = rc;
      job->res.rank = rank;
      job->res.end_ms = s->now_ms();
      job->state = 2;
      s->groups_used -= job->groups;
      s->give(off, job->ws);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  if (st) hipStreamDestroy(st);
}

}  // namespace
}  // namespace qrcp

extern "C" {

qrcp_server* qrcp_server_create(const qrcp_server_cfg* cfg) {
  qrcp_server_cfg c{};
  c.struct_size = sizeof(qrcp_server_cfg);
  if (cfg) c = *cfg;
  if (c.slots < 0 || c.slots > 64 || c.hbm_budget < 0) return nullptr;
  int dev = c.device;
  if (hipSetDevice(dev) != hipSuccess) return nullptr;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return nullptr;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return nullptr;
  qrcp_server* s = new qrcp_server();
  s->device = dev;
  s->slots = c.slots ? c.slots : 8;
  s->budget = c.hbm_budget ? c.hbm_budget
                           : std::min<int64_t>((int64_t)(0.8 * (double)free_b), int64_t(4) << 30);
  s->budget = s->budget / 256 * 256;
  s->cu_budget = cus;
  // the whole pool up front: requests only take and return slices of it
  void* pool = nullptr;
  if (s->budget <= 0 || hipMalloc(&pool, (size_t)s->budget) != hipSuccess) {
    delete s;
    return nullptr;
  }
  s->pool = (char*)pool;
  s->free_list[0] = (size_t)s->budget;
  s->t0 = std::chrono::steady_clock::now();
  for (int w = 0; w < s->slots; ++w) s->workers.emplace_back(qrcp::worker_main, s, w);
  return s;
}

int qrcp_server_submit(qrcp_server* s, const qrcp_request* req, uint64_t* ticket) {
  if (!s) return -1;
  if (!req || req->struct_size != (int32_t)sizeof(qrcp_request)) return -2;
  if (!ticket) return -3;
  const qrcp_request& r = *req;
  if (r.m < 0 || r.n < 0 || r.lda < std::max<int64_t>(1, r.m) || r.block_size < 1 ||
      !(r.sketch_factor >= 1.0) || !(r.tol >= 0.0) || (!r.A && r.m * r.n > 0))
    return -2;
  // the same up-front limits as qrcp_factor: sketch rows and the pivot
  // selection's resident grid for the first block
  if (r.n > 0 && (std::ceil(r.sketch_factor * (double)r.block_size - 1e-12) > 1024.0 ||
                  qrcp::lu_resident_groups(r.n) == 0))
    return QRCP_ERR_UNSUPPORTED;
  const size_t ws = qrcp_workspace_size(r.m, r.n, r.block_size, r.sketch_factor, &r.opts);
  const int groups = qrcp::request_groups(r);
  if ((int64_t)ws > s->budget || groups > s->cu_budget) return QRCP_ERR_UNSUPPORTED;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return -1;
    const uint64_t id = s->next++;
    qrcp_server::Job& j = s->jobs[id];
    j.req = r;
    j.res = qrcp_result{};
    j.res.struct_size = sizeof(qrcp_result);
    j.res.submit_ms = s->now_ms();
    j.ws = ws;
    j.groups = groups;
    s->queue.push_back(id);
    *ticket = id;
  }
  s->cv_work.notify_all();
  return QRCP_OK;
}

int qrcp_server_poll(qrcp_server* s, uint64_t ticket, qrcp_result* out) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return -2;
  if (it->second.state != 2) return 1;
  if (out) *out = it->second.res;
  s->jobs.erase(it);
  return 0;
}

int qrcp_server_wait(qrcp_server* s, uint64_t ticket, qrcp_result* out) {
  if (!s) return -1;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return -2;
  s->cv_done.wait(lk, [&] { return it->second.state == 2; });
  if (out) *out = it->second.res;
  s->jobs.erase(it);
  return 0;
}

int qrcp_server_pending(qrcp_server* s) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  int n = 0;
  for (auto& kv : s->jobs) n += kv.second.state != 2;
  return n;
}

void qrcp_server_destroy(qrcp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  if (s->pool) (void)hipFree(s->pool);
  delete s;
}

}  // extern "C"
