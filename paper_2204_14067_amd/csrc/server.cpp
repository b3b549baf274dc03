// Request loop with admission by HBM footprint (bmg_server_* of bmg.h).
//
// A request is a host copy of one completion problem plus its options.  The
// server keeps a FIFO of queued requests; a slot takes the first queued
// request whose footprint fits a first-fit allocation of the caller's device
// arena, copies its CSR to the device, creates the problem and solves it on
// the slot's own HIP stream, copies the factors back and releases the memory.
// Two ways to drive the slots:
//   - threads: one host worker per slot runs each solve to the end; while
//     solving, each problem is attached to the server's pass batcher, so the
//     sparse passes of the running problems that are pending at the same
//     time share one launch (batch.h);
//   - tick: no threads; every bmg_server_tick call on the caller's thread
//     admits what fits and advances each running solve by one outer
//     iteration of Algorithm 1 (round robin over the slots' streams).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "bmg.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
size_t rup(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Request {
  uint64_t id = 0;
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int k_cap = 0, ld = 0;
  bmg_precision prec = BMG_FP32;
  bmg_options opt{};
  size_t ws_bytes = 0, footprint = 0, off = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
  bmg_status status = BMG_OK;
  // tick mode: the running solve
  bmg_problem *P = nullptr;
  bmg::SolveTask *task = nullptr;
  double *d_W = nullptr, *d_H = nullptr;
  int slot = -1;
  int k = 0;
  bmg_result res{};
  std::vector<double> W, H;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

size_t ld_for(int k_cap) { return rup((size_t)std::max(k_cap, 1), 8); }

bmg_status footprint(int64_t m, int64_t n, int64_t nnz, int k_cap, bmg_precision prec,
                     const bmg_options *opt, size_t *ws, size_t *total) {
  size_t w = 0;
  bmg_status st = bmg_workspace_size(m, n, nnz, k_cap, prec, opt, &w);
  if (st != BMG_OK) return st;
  const size_t ld = ld_for(k_cap);
  *ws = w;
  *total = rup(8 * (m + 1), 256) + rup(4 * std::max<int64_t>(nnz, 1), 256) +
           rup(8 * std::max<int64_t>(nnz, 1), 256) + rup(8 * m * ld, 256) + rup(8 * n * ld, 256) +
           rup(w, 256);
  return BMG_OK;
}

}  // namespace

struct bmg_server {
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;       // queue / free memory changed
  std::condition_variable done_cv;  // a request finished
  std::deque<Request *> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted, coalesced
  std::vector<std::thread> workers;
  // tick mode: slot streams and the requests running in them
  bool tick_mode = false;
  std::vector<hipStream_t> streams;
  std::vector<Request *> slots;
  bool stop = false;
  uint64_t next_id = 1;
  int running = 0, peak_running = 0;
  size_t used = 0, peak_used = 0;
  int outstanding = 0;
  bmg::PassBatcher *batcher = nullptr;

  bool alloc(size_t bytes, size_t *off) {
    for (size_t i = 0; i < free_list.size(); ++i) {
      if (free_list[i].second >= bytes) {
        *off = free_list[i].first;
        free_list[i].first += bytes;
        free_list[i].second -= bytes;
        if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
        used += bytes;
        peak_used = std::max(peak_used, used);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used -= bytes;
    auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
    it = free_list.insert(it, {off, bytes});
    size_t i = it - free_list.begin();
    if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
      free_list[i].second += free_list[i + 1].second;
      free_list.erase(free_list.begin() + i + 1);
    }
    if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
      free_list[i - 1].second += free_list[i].second;
      free_list.erase(free_list.begin() + i);
    }
  }
  // first queued request (arrival order) whose footprint fits now
  Request *admit_locked() {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      size_t off;
      if (alloc((*it)->footprint, &off)) {
        Request *r = *it;
        r->off = off;
        queue.erase(it);
        return r;
      }
    }
    return nullptr;
  }
  bmg_status start(Request *r, hipStream_t st);
  void finish(Request *r, hipStream_t st, bmg_status s);
  void run(Request *r, hipStream_t st);
  void worker();
  void admitted_locked(Request *r) {
    r->state = 1;
    r->t_admit = now_s();
    running += 1;
    peak_running = std::max(peak_running, running);
  }
  void retire_locked(Request *r) {
    r->t_done = now_s();
    r->state = (r->status >= 0) ? 2 : 3;
    release(r->off, r->footprint);
    running -= 1;
    outstanding -= 1;
  }
};

// Copies the request's CSR into its arena block and creates the problem and
// the solve (the initialisation runs here); r->P / r->task are set on success.
bmg_status bmg_server::start(Request *r, hipStream_t st) {
  char *base = arena + r->off;
  size_t o = 0;
  auto take = [&](size_t bytes) { char *p = base + o; o += rup(bytes, 256); return p; };
  int64_t *d_rp = (int64_t *)take(8 * (r->m + 1));
  int32_t *d_col = (int32_t *)take(4 * std::max<int64_t>(r->nnz, 1));
  double *d_val = (double *)take(8 * std::max<int64_t>(r->nnz, 1));
  r->d_W = (double *)take(8 * r->m * r->ld);
  r->d_H = (double *)take(8 * r->n * r->ld);
  void *ws = take(r->ws_bytes);
  bool ok = hipMemcpyAsync(d_rp, r->row_ptr.data(), 8 * (r->m + 1), hipMemcpyHostToDevice, st) == hipSuccess;
  if (r->nnz > 0) {
    ok = ok && hipMemcpyAsync(d_col, r->col.data(), 4 * r->nnz, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(d_val, r->val.data(), 8 * r->nnz, hipMemcpyHostToDevice, st) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  // host copies of the input are no longer needed
  std::vector<int64_t>().swap(r->row_ptr);
  std::vector<int32_t>().swap(r->col);
  std::vector<double>().swap(r->val);
  if (!ok) return BMG_EDEVICE;
  bmg_csr csr{r->m, r->n, r->nnz, d_rp, d_col, d_val};
  bmg_status s = bmg_problem_create(&csr, r->k_cap, r->prec, &r->opt, ws, r->ws_bytes, st, &r->P);
  if (s != BMG_OK) return s;
  if (!tick_mode) bmg::batcher_attach(r->P, batcher);
  s = bmg::solve_task_create(r->P, &r->opt, &r->task);
  return s;
}

// Final objective and factors of the solve (status s so far), copied back to
// the host; the problem and the task are released.
void bmg_server::finish(Request *r, hipStream_t st, bmg_status s) {
  if (s == BMG_OK && r->task) {
    int k = 0;
    s = bmg::solve_task_finish(r->task, r->d_W, r->d_H, r->ld, &k, &r->res);
    r->k = k;
    if (s >= 0) {
      r->W.resize((size_t)r->m * r->ld);
      r->H.resize((size_t)r->n * r->ld);
      const bool ok =
          hipMemcpyAsync(r->W.data(), r->d_W, 8 * r->m * r->ld, hipMemcpyDeviceToHost, st) == hipSuccess &&
          hipMemcpyAsync(r->H.data(), r->d_H, 8 * r->n * r->ld, hipMemcpyDeviceToHost, st) == hipSuccess &&
          hipStreamSynchronize(st) == hipSuccess;
      if (!ok) s = BMG_EDEVICE;
    }
  }
  if (r->task) bmg::solve_task_destroy(r->task);
  r->task = nullptr;
  if (r->P) {
    if (!tick_mode) bmg::batcher_detach(r->P);
    bmg_problem_destroy(r->P);
  }
  r->P = nullptr;
  r->status = s;
}

void bmg_server::run(Request *r, hipStream_t st) {
  bmg_status s = start(r, st);
  int done = 0;
  while (s == BMG_OK && !done) s = bmg::solve_task_step(r->task, &done);
  finish(r, st, s);
}

void bmg_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  if (hipStreamCreate(&st) != hipSuccess) st = nullptr;
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        if (stop) return true;
        if (queue.empty()) return false;
        r = admit_locked();
        return r != nullptr;
      });
      if (!r) break;  // stop requested
      admitted_locked(r);
    }
    run(r, st);
    {
      std::lock_guard<std::mutex> lk(mu);
      retire_locked(r);
    }
    cv.notify_all();
    done_cv.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

extern "C" bmg_status bmg_server_footprint(int64_t m, int64_t n, int64_t nnz, int k_cap,
                                           bmg_precision prec, const bmg_options *opt, size_t *bytes) {
  size_t ws = 0;
  if (!bytes) return BMG_EINVAL;
  return footprint(m, n, nnz, k_cap, prec, opt, &ws, bytes);
}

extern "C" bmg_status bmg_server_create(void *arena, size_t arena_bytes, int max_slots, int threads,
                                        bmg_server **out) {
  if (!arena || !out || arena_bytes < 4096 || max_slots < 1 || max_slots > 64 ||
      (threads != 0 && threads != 1))
    return BMG_EINVAL;
  bmg_server *S = new bmg_server();
  S->arena = (char *)arena;
  S->arena_bytes = arena_bytes;
  S->free_list.push_back({0, arena_bytes / 256 * 256});
  (void)hipGetDevice(&S->device);
  S->tick_mode = threads == 0;
  if (S->tick_mode) {
    for (int i = 0; i < max_slots; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreate(&st) != hipSuccess) {
        for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
        delete S;
        return BMG_EDEVICE;
      }
      S->streams.push_back(st);
    }
    S->slots.assign(max_slots, nullptr);
  } else {
    S->batcher = bmg::batcher_create();
    if (!S->batcher) {
      delete S;
      return BMG_EDEVICE;
    }
    for (int i = 0; i < max_slots; ++i) S->workers.emplace_back([S] { S->worker(); });
  }
  *out = S;
  return BMG_OK;
}

extern "C" bmg_status bmg_server_tick(bmg_server *S, int *running, int *queued) {
  if (!S) return BMG_EINVAL;
  if (S->tick_mode) {
    // admit into free slots, in arrival order with backfill
    for (size_t i = 0; i < S->slots.size(); ++i) {
      if (S->slots[i]) continue;
      Request *r = nullptr;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->queue.empty()) r = S->admit_locked();
        if (r) S->admitted_locked(r);
      }
      if (!r) break;
      r->slot = (int)i;
      S->slots[i] = r;
      const bmg_status s = S->start(r, S->streams[i]);
      if (s != BMG_OK) {
        S->finish(r, S->streams[i], s);
        std::lock_guard<std::mutex> lk(S->mu);
        S->retire_locked(r);
        S->slots[i] = nullptr;
        S->done_cv.notify_all();
      }
    }
    // one outer iteration of every running solve
    for (size_t i = 0; i < S->slots.size(); ++i) {
      Request *r = S->slots[i];
      if (!r) continue;
      int done = 0;
      const bmg_status s = bmg::solve_task_step(r->task, &done);
      if (s != BMG_OK || done) {
        S->finish(r, S->streams[i], s);
        std::lock_guard<std::mutex> lk(S->mu);
        S->retire_locked(r);
        S->slots[i] = nullptr;
        S->done_cv.notify_all();
      }
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (running) *running = S->running;
  if (queued) *queued = (int)S->queue.size();
  return BMG_OK;
}

extern "C" bmg_status bmg_server_submit(bmg_server *S, const bmg_csr *c, int k_cap,
                                        bmg_precision prec, const bmg_options *opt,
                                        uint64_t *ticket) {
  if (!S || !c || !opt || !ticket || c->m <= 0 || c->n <= 0 || c->nnz < 0) return BMG_EINVAL;
  if (c->nnz > 0 && (!c->row_ptr || !c->col || !c->val)) return BMG_EINVAL;
  std::unique_ptr<Request> r(new Request());
  r->m = c->m; r->n = c->n; r->nnz = c->nnz;
  r->k_cap = k_cap;
  r->ld = (int)ld_for(k_cap);
  r->prec = prec;
  r->opt = *opt;
  // the workspace holds the request's own variants (history blocks, SpaRSA state)
  bmg_status st = footprint(c->m, c->n, c->nnz, k_cap, prec, opt, &r->ws_bytes, &r->footprint);
  if (st != BMG_OK) return st;
  if (r->footprint > S->arena_bytes) return BMG_ENOMEM;
  r->row_ptr.assign(c->row_ptr, c->row_ptr + c->m + 1);
  r->col.assign(c->col, c->col + c->nnz);
  r->val.assign(c->val, c->val + c->nnz);
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->id = S->next_id++;
    *ticket = r->id;
    S->queue.push_back(r.get());
    S->outstanding += 1;
    S->reqs[r->id] = std::move(r);
  }
  S->cv.notify_all();
  return BMG_OK;
}

extern "C" bmg_status bmg_server_poll(bmg_server *S, uint64_t ticket, bmg_request_info *info,
                                      double *W_host, double *H_host, int ld) {
  if (!S || !info) return BMG_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return BMG_EINVAL;
  Request *r = it->second.get();
  memset(info, 0, sizeof(*info));
  info->state = r->state;
  info->footprint = r->footprint;
  if (r->state >= 2) {
    info->status = r->status;
    info->k = r->k;
    info->queued_s = r->t_admit - r->t_submit;
    info->run_s = r->t_done - r->t_admit;
    info->total_s = r->t_done - r->t_submit;
    info->result = r->res;
    if (r->state == 2 && W_host && H_host) {
      if (ld < r->k) return BMG_EINVAL;
      for (int64_t i = 0; i < r->m; ++i)
        for (int j = 0; j < ld; ++j)
          W_host[i * ld + j] = (j < r->ld && j < r->k) ? r->W[i * r->ld + j] : 0.0;
      for (int64_t i = 0; i < r->n; ++i)
        for (int j = 0; j < ld; ++j)
          H_host[i * ld + j] = (j < r->ld && j < r->k) ? r->H[i * r->ld + j] : 0.0;
    }
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_server_drain(bmg_server *S) {
  if (!S) return BMG_EINVAL;
  if (S->tick_mode) {
    for (;;) {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->outstanding == 0) return BMG_OK;
      }
      bmg_status s = bmg_server_tick(S, nullptr, nullptr);
      if (s != BMG_OK) return s;
    }
  }
  std::unique_lock<std::mutex> lk(S->mu);
  S->done_cv.wait(lk, [&] { return S->outstanding == 0; });
  return BMG_OK;
}

extern "C" bmg_status bmg_server_stats(bmg_server *S, int *peak_running, size_t *peak_bytes) {
  if (!S) return BMG_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (peak_running) *peak_running = S->peak_running;
  if (peak_bytes) *peak_bytes = S->peak_used;
  return BMG_OK;
}

extern "C" bmg_status bmg_server_batch_stats(bmg_server *S, int64_t *launches, int64_t *passes) {
  if (!S) return BMG_EINVAL;
  long l = 0, p = 0;
  bmg::batcher_stats(S->batcher, &l, &p);
  if (launches) *launches = l;
  if (passes) *passes = p;
  return BMG_OK;
}

extern "C" void bmg_server_destroy(bmg_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Request *r : S->queue) {
      r->state = 3;
      r->status = BMG_ECANCELLED;
      S->outstanding -= 1;
    }
    S->queue.clear();
  }
  S->cv.notify_all();
  for (auto &t : S->workers) t.join();
  // tick mode: running solves end here, their results are dropped
  for (size_t i = 0; i < S->slots.size(); ++i) {
    Request *r = S->slots[i];
    if (!r) continue;
    if (r->task) bmg::solve_task_destroy(r->task);
    if (r->P) bmg_problem_destroy(r->P);
    S->slots[i] = nullptr;
  }
  for (hipStream_t x : S->streams) {
    (void)hipStreamSynchronize(x);
    (void)hipStreamDestroy(x);
  }
  if (S->batcher) bmg::batcher_destroy(S->batcher);
  delete S;
}
