// Request loop over one index: continuous, size-adaptive batching (the
// serving form of the appendix's "Batch Inference": requests are bundled so
// that one scan of the corpus answers a whole batch).
//
// Threads: callers queue requests (fr_server_submit); one dispatcher forms a
// batch of everything pending whenever fewer than max_inflight batches are on
// the device and enqueues it on the server's stream; one completion thread
// waits for batches in order and copies their rows to the callers' buffers.
// All device and pinned memory is allocated in fr_server_create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "fr.h"
#include "fr_host.h"

using namespace fr;

namespace {

constexpr uint32_t kFailed = 0xFFFFFFFFu;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t ticket = 0;
  uint64_t t_arr = 0;
  uint32_t k = 0;
  uint32_t n_lits = 0;
  std::vector<float> emb;
  std::vector<uint32_t> clause_len;  // literals of each clause
  std::vector<uint32_t> lits;
  uint32_t* ids = nullptr;
  float* scores = nullptr;
  uint32_t* count = nullptr;
  uint64_t* nmatch = nullptr;
  uint64_t* done_ns = nullptr;
  int32_t* status = nullptr;
};

// One batch's buffers: device inputs / outputs and their pinned twins.
struct Slot {
  float* d_q = nullptr;
  uint32_t* d_ids = nullptr;
  float* d_scores = nullptr;
  uint32_t* d_count = nullptr;
  uint64_t* d_nm = nullptr;
  float* h_q = nullptr;
  uint32_t* h_ids = nullptr;
  float* h_scores = nullptr;
  uint32_t* h_count = nullptr;
  uint64_t* h_nm = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Req> reqs;
  fr_status st = FR_OK;
  bool busy = false;
};

}  // namespace

struct fr_server {
  fr_index* ix = nullptr;
  IndexShape sh{};
  uint32_t max_batch = 0, max_inflight = 0, max_wait_us = 0;
  hipStream_t stream = nullptr;
  std::vector<Slot> slots;
  std::deque<Req> pending;
  std::deque<Slot*> inflight;
  std::mutex mu;
  std::condition_variable cv_disp, cv_comp, cv_done;
  uint64_t next_ticket = 0, completed = 0;
  bool stop = false, disp_exited = false;
  std::thread disp, comp;
  fr_server_stats stats{};
};

namespace {

void release(fr_server* sv) {
  for (Slot& s : sv->slots) {
    for (void* p : {(void*)s.d_q, (void*)s.d_ids, (void*)s.d_scores, (void*)s.d_count,
                    (void*)s.d_nm})
      if (p) (void)hipFree(p);
    for (void* p : {(void*)s.h_q, (void*)s.h_ids, (void*)s.h_scores, (void*)s.h_count,
                    (void*)s.h_nm})
      if (p) (void)hipHostFree(p);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  sv->slots.clear();
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  sv->stream = nullptr;
}

Slot* free_slot(fr_server* sv) {
  for (Slot& s : sv->slots)
    if (!s.busy) return &s;
  return nullptr;
}

// Enqueue one batch on the server's stream: queries up, the search, rows
// down, the batch's event.  Returns the first failing status.
fr_status enqueue_batch(fr_server* sv, Slot& sl, std::vector<uint32_t>& co,
                        std::vector<uint32_t>& lo, std::vector<uint32_t>& terms,
                        std::vector<uint32_t>& kk) {
  const uint32_t n = (uint32_t)sl.reqs.size();
  const uint32_t d = sv->sh.dim, km = sv->sh.k_max;
  co.assign(1, 0);
  lo.assign(1, 0);
  terms.clear();
  kk.clear();
  for (uint32_t i = 0; i < n; ++i) {
    const Req& r = sl.reqs[i];
    std::memcpy(sl.h_q + (size_t)i * d, r.emb.data(), (size_t)d * 4);
    for (uint32_t len : r.clause_len) lo.push_back(lo.back() + len);
    co.push_back(co.back() + (uint32_t)r.clause_len.size());
    terms.insert(terms.end(), r.lits.begin(), r.lits.end());
    kk.push_back(r.k);
  }
  if (hipMemcpyAsync(sl.d_q, sl.h_q, (size_t)n * d * 4, hipMemcpyHostToDevice, sv->stream) !=
      hipSuccess)
    return set_error(FR_EDEVICE, "server: query copy failed");
  const fr_cnf_batch cnf{n, co.data(), lo.data(), terms.data()};
  const fr_status st = fr_search(sv->ix, n, sl.d_q, &cnf, kk.data(), sl.d_ids, sl.d_scores,
                                 sl.d_count, sl.d_nm, sv->stream, FR_DEVICE_PTRS);
  if (st != FR_OK) return st;
  if (hipMemcpyAsync(sl.h_ids, sl.d_ids, (size_t)n * km * 4, hipMemcpyDeviceToHost,
                     sv->stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_scores, sl.d_scores, (size_t)n * km * 4, hipMemcpyDeviceToHost,
                     sv->stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_count, sl.d_count, (size_t)n * 4, hipMemcpyDeviceToHost,
                     sv->stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_nm, sl.d_nm, (size_t)n * 8, hipMemcpyDeviceToHost, sv->stream) !=
          hipSuccess ||
      hipEventRecord(sl.done, sv->stream) != hipSuccess)
    return set_error(FR_EDEVICE, "server: result copy failed");
  return FR_OK;
}

void dispatch_loop(fr_server* sv) {
  (void)hipSetDevice(sv->sh.device);
  std::vector<uint32_t> co, lo, terms, kk;
  std::unordered_set<uint32_t> dict;
  for (;;) {
    Slot* sl = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        if (sv->stop && sv->pending.empty()) {
          sv->disp_exited = true;
          sv->cv_comp.notify_all();
          return;
        }
        sl = free_slot(sv);
        if (sl && !sv->pending.empty()) break;
        sv->cv_disp.wait(lk);
      }
      // an idle device may wait a little for a fuller batch
      if (sv->max_wait_us && sv->inflight.empty() && !sv->stop &&
          sv->pending.size() < sv->max_batch) {
        const uint64_t until_ns = sv->pending.front().t_arr + sv->max_wait_us * 1000ull;
        const auto until = std::chrono::steady_clock::time_point(
            std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                std::chrono::nanoseconds(until_ns)));
        sv->cv_disp.wait_until(
            lk, until, [&] { return sv->stop || sv->pending.size() >= sv->max_batch; });
      }
      // requests in submission order, within one search's limits (each
      // request alone fits: fr_server_submit checked it); with term lists
      // also within the batch's distinct-term limit
      uint32_t nc = 0, nl = 0;
      dict.clear();
      while (!sv->pending.empty() && sl->reqs.size() < sv->max_batch) {
        const Req& r = sv->pending.front();
        if (!sl->reqs.empty() && (nc + r.clause_len.size() > sv->sh.max_clauses ||
                                  nl + r.n_lits > sv->sh.max_literals))
          break;
        if (sv->sh.batch_terms) {
          size_t fresh = 0;
          for (uint32_t t : r.lits) fresh += !dict.count(t);
          if (!sl->reqs.empty() && dict.size() + fresh > sv->sh.batch_terms) break;
          dict.insert(r.lits.begin(), r.lits.end());
        }
        nc += (uint32_t)r.clause_len.size();
        nl += r.n_lits;
        sl->reqs.push_back(std::move(sv->pending.front()));
        sv->pending.pop_front();
      }
      sl->busy = true;
    }
    sl->st = enqueue_batch(sv, *sl, co, lo, terms, kk);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      const uint32_t n = (uint32_t)sl->reqs.size();
      sv->stats.batches += 1;
      sv->stats.queries += n;
      if (n > sv->stats.max_batch_seen) sv->stats.max_batch_seen = n;
      sv->inflight.push_back(sl);
      sv->cv_comp.notify_one();
    }
  }
}

void complete_loop(fr_server* sv) {
  (void)hipSetDevice(sv->sh.device);
  const uint32_t km = sv->sh.k_max;
  for (;;) {
    Slot* sl = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_comp.wait(lk, [&] { return !sv->inflight.empty() || sv->disp_exited; });
      if (sv->inflight.empty()) return;
      sl = sv->inflight.front();
    }
    fr_status st = sl->st;
    if (st == FR_OK && hipEventSynchronize(sl->done) != hipSuccess) st = FR_EDEVICE;
    const uint64_t t = now_ns();
    uint64_t n_failed = 0;
    for (size_t i = 0; i < sl->reqs.size(); ++i) {
      Req& r = sl->reqs[i];
      int32_t rs = st;
      if (st == FR_OK) {
        std::memcpy(r.ids, sl->h_ids + i * km, (size_t)km * 4);
        std::memcpy(r.scores, sl->h_scores + i * km, (size_t)km * 4);
        *r.count = sl->h_count[i];
        *r.nmatch = sl->h_nm[i];
        if (sl->h_count[i] == kFailed) rs = FR_EUNSUPPORTED;
      } else {
        for (uint32_t j = 0; j < km; ++j) {
          r.ids[j] = kFailed;
          r.scores[j] = -INFINITY;
        }
        *r.count = kFailed;
        *r.nmatch = 0;
      }
      if (r.status) *r.status = rs;
      if (r.done_ns) *r.done_ns = t;
      n_failed += rs != FR_OK;
    }
    const uint64_t last = sl->reqs.back().ticket;
    sl->reqs.clear();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->inflight.pop_front();
      sl->busy = false;
      sv->completed = last + 1;
      sv->stats.failed += n_failed;
      sv->cv_done.notify_all();
      sv->cv_disp.notify_one();
    }
  }
}

}  // namespace

extern "C" {

uint64_t fr_clock_ns(void) { return now_ns(); }

fr_status fr_server_create(fr_index* ix, const fr_server_config* cfg, fr_server** out) {
  if (!ix || !cfg || !out) return set_error(FR_EINVAL, "null argument");
  *out = nullptr;
  IndexShape sh{};
  fr_status st = index_shape(ix, &sh);
  if (st != FR_OK) return st;
  const uint32_t mb = cfg->max_batch ? cfg->max_batch : sh.max_batch;
  const uint32_t mi = cfg->max_inflight ? cfg->max_inflight : std::min(2u, sh.n_workspaces);
  if (mb < 1 || mb > sh.max_batch)
    return set_error(FR_EINVAL, "server max_batch must be 1..the index's max_batch (" +
                                    std::to_string(sh.max_batch) + ")");
  if (mi < 1 || mi > sh.n_workspaces)
    return set_error(FR_EINVAL, "server max_inflight must be 1..the index's n_workspaces (" +
                                    std::to_string(sh.n_workspaces) + ")");
  if (hipSetDevice(sh.device) != hipSuccess) return set_error(FR_EDEVICE, "hipSetDevice failed");
  std::unique_ptr<fr_server> sv(new fr_server);
  sv->ix = ix;
  sv->sh = sh;
  sv->max_batch = mb;
  sv->max_inflight = mi;
  sv->max_wait_us = cfg->max_wait_us;
  if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
    sv->stream = nullptr;
    return set_error(FR_EDEVICE, "hipStreamCreate failed");
  }
  sv->slots.resize(mi);
  const size_t rows = (size_t)mb * sh.k_max;
  bool ok = true;
  for (Slot& s : sv->slots) {
    ok = ok && hipMalloc((void**)&s.d_q, (size_t)mb * sh.dim * 4) == hipSuccess;
    ok = ok && hipMalloc((void**)&s.d_ids, rows * 4) == hipSuccess;
    ok = ok && hipMalloc((void**)&s.d_scores, rows * 4) == hipSuccess;
    ok = ok && hipMalloc((void**)&s.d_count, (size_t)mb * 4) == hipSuccess;
    ok = ok && hipMalloc((void**)&s.d_nm, (size_t)mb * 8) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s.h_q, (size_t)mb * sh.dim * 4, hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipHostMalloc((void**)&s.h_ids, rows * 4, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s.h_scores, rows * 4, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s.h_count, (size_t)mb * 4, hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipHostMalloc((void**)&s.h_nm, (size_t)mb * 8, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    release(sv.get());
    return set_error(FR_ENOMEM, "server buffers could not be allocated");
  }
  fr_server* p = sv.get();
  p->disp = std::thread(dispatch_loop, p);
  p->comp = std::thread(complete_loop, p);
  *out = sv.release();
  return FR_OK;
}

fr_status fr_server_submit(fr_server* sv, uint32_t n, const float* queries,
                           const fr_cnf_batch* cnf, const uint32_t* k,
                           const uint64_t* t_arrival_ns, uint32_t* out_ids, float* out_scores,
                           uint32_t* out_count, uint64_t* out_nmatch, uint64_t* out_done_ns,
                           int32_t* out_status, uint64_t* out_first_ticket) {
  if (!sv || !cnf) return set_error(FR_EINVAL, "null argument");
  if (cnf->n_queries != n) return set_error(FR_EINVAL, "cnf->n_queries != n");
  if (n == 0) return FR_OK;
  if (!queries || !k || !cnf->clause_off || !out_ids || !out_scores || !out_count || !out_nmatch)
    return set_error(FR_EINVAL, "null query, predicate or output pointer");
  const IndexShape& sh = sv->sh;
  const uint32_t n_c = cnf->clause_off[n];
  if (cnf->clause_off[0] != 0 || (n_c && (!cnf->literal_off || cnf->literal_off[0] != 0)))
    return set_error(FR_EINVAL, "clause_off[0] and literal_off[0] must be 0");
  if (n_c && cnf->literal_off[n_c] && !cnf->terms) return set_error(FR_EINVAL, "terms missing");
  std::vector<Req> reqs(n);
  const uint64_t t0 = now_ns();
  for (uint32_t q = 0; q < n; ++q) {
    const uint32_t c0 = cnf->clause_off[q], c1 = cnf->clause_off[q + 1];
    if (c1 < c0) return set_error(FR_EINVAL, "clause_off must be non-decreasing");
    if (k[q] > sh.k_max) return set_error(FR_EINVAL, "k exceeds k_max");
    Req& r = reqs[q];
    r.k = k[q];
    r.t_arr = t_arrival_ns ? t_arrival_ns[q] : t0;
    r.emb.assign(queries + (size_t)q * sh.dim, queries + (size_t)(q + 1) * sh.dim);
    for (uint32_t c = c0; c < c1; ++c) {
      const uint32_t l0 = cnf->literal_off[c], l1 = cnf->literal_off[c + 1];
      if (l1 < l0) return set_error(FR_EINVAL, "literal_off must be non-decreasing");
      for (uint32_t l = l0; l < l1; ++l)
        if (cnf->terms[l] >= sh.vocab)
          return set_error(FR_EINVAL, "term id " + std::to_string(cnf->terms[l]) + " >= vocab");
      r.clause_len.push_back(l1 - l0);
      r.lits.insert(r.lits.end(), cnf->terms + l0, cnf->terms + l1);
    }
    r.n_lits = (uint32_t)r.lits.size();
    if (r.clause_len.size() > sh.max_clauses || r.n_lits > sh.max_literals)
      return set_error(FR_EINVAL, "request " + std::to_string(q) +
                                      " has more clauses or literals than one search takes");
    if (sh.batch_terms) {
      std::vector<uint32_t> u(r.lits);
      std::sort(u.begin(), u.end());
      if ((size_t)(std::unique(u.begin(), u.end()) - u.begin()) > sh.batch_terms)
        return set_error(FR_EINVAL, "request " + std::to_string(q) +
                                        " has more distinct terms than one search takes");
    }
    r.ids = out_ids + (size_t)q * sh.k_max;
    r.scores = out_scores + (size_t)q * sh.k_max;
    r.count = out_count + q;
    r.nmatch = out_nmatch + q;
    r.done_ns = out_done_ns ? out_done_ns + q : nullptr;
    r.status = out_status ? out_status + q : nullptr;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) return set_error(FR_EINVAL, "the server is shutting down");
  if (out_first_ticket) *out_first_ticket = sv->next_ticket;
  for (Req& r : reqs) {
    r.ticket = sv->next_ticket++;
    sv->pending.push_back(std::move(r));
  }
  sv->cv_disp.notify_one();
  return FR_OK;
}

fr_status fr_server_wait(fr_server* sv, uint64_t ticket, uint32_t timeout_ms) {
  if (!sv) return set_error(FR_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (ticket >= sv->next_ticket) return set_error(FR_EINVAL, "ticket was never issued");
  auto done = [&] { return sv->completed > ticket; };
  if (timeout_ms == 0xFFFFFFFFu) {
    sv->cv_done.wait(lk, done);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    return set_error(FR_EBUSY, "timed out waiting for ticket " + std::to_string(ticket));
  }
  return FR_OK;
}

fr_status fr_server_get_stats(fr_server* sv, fr_server_stats* out) {
  if (!sv || !out) return set_error(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  out->pending = (uint32_t)sv->pending.size();
  return FR_OK;
}

fr_status fr_server_destroy(fr_server* sv) {
  if (!sv) return FR_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv_disp.notify_all();
  }
  if (sv->disp.joinable()) sv->disp.join();
  if (sv->comp.joinable()) sv->comp.join();
  if (sv->stream) (void)hipStreamSynchronize(sv->stream);
  release(sv);
  delete sv;
  return FR_OK;
}

}  // extern "C"
