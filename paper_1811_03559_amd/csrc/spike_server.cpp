// Serving runtime: continuous batching of banded solves on one GPU.
//
// Requests name a matrix by an id chosen by the caller.  The first request
// for an id factors the matrix into a workspace carved from the server's
// device pool (hbm_budget bytes of device memory the caller allocates and
// passes in; the server allocates no device memory itself); later
// requests for the id reuse the resident factorisation.  Resident
// factorisations are evicted least-recently-used, when idle, to make room.
// A worker thread admits pending requests while request slots and pool
// memory are free, gives every matrix a home stream (all work on one
// factorisation is ordered on it, since the solves share its workspace), and
// on every scheduling pass launches the admitted solves homed on one stream
// as one batched solve (spike_solve_batch).  Completion is observed with an
// event per request; latency is measured from submission to the observed
// completion on the host clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/spike.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap) with 256-byte granules.
class Pool {
 public:
  explicit Pool(size_t cap) : cap_(cap) { free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, o = it->first;
        free_.erase(it);
        if (rest) free_[o + bytes] = rest;
        used_ += bytes;
        hwm_ = std::max(hwm_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
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
  size_t used() const { return used_; }
  size_t hwm() const { return hwm_; }
  size_t cap() const { return cap_; }

 private:
  size_t cap_, used_ = 0, hwm_ = 0;
  std::map<size_t, size_t> free_;
};

struct Resident {
  int64_t id;
  int64_t n = 0;               // the matrix it was factored from
  int32_t kl = 0, ku = 0;
  const double* dAB = nullptr;
  spike_handle h = nullptr;
  size_t off = 0, bytes = 0;
  int stream = 0;
  hipEvent_t last = nullptr;   // after the latest work on this factorisation
  int pending = 0;             // admitted requests not completed yet
  uint64_t last_use = 0;
  bool info_known = false;     // numerical status read once, after the factorisation
  int64_t info = 0;
  const spike_request* freq = nullptr;   // its factorisation waits for this pass's batch
};

struct Req {
  int64_t ticket;
  spike_request r;
  double t_arrive = 0, t_done = 0;
  int state = 0;   // 0 pending, 1 on the device, 2 done, 3 failed
  int err = 0;
  int64_t info = 0;   // numerical status of the factorisation (spike_info)
  hipEvent_t done = nullptr;
  Resident* res = nullptr;
};

}  // namespace

struct spike_server_s {
  uint32_t magic = 0;
  spike_server_opts o;
  char* base = nullptr;
  Pool* pool = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<int> load;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::vector<Req*> inflight;
  std::unordered_map<int64_t, Req*> reqs;
  std::unordered_map<int64_t, Resident*> res;
  std::map<int, std::vector<Resident*>> deferred;   // new factorisations of a pass, per stream
  std::vector<hipEvent_t> event_pool;
  std::vector<double> lat;
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  int64_t factorizations = 0, evictions = 0, completed = 0, failed = 0;
  double t_first = 0, t_last = 0;
  bool stop = false;
  int device = 0;
  std::thread worker;

  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  // Evicts idle residents (LRU first) until `bytes` fit; true if they fit.
  bool make_room(size_t bytes, size_t* off) {
    while (!pool->alloc(bytes, off)) {
      Resident* victim = nullptr;
      for (auto& kv : res) {
        Resident* r = kv.second;
        if (r->pending > 0) continue;
        if (r->last && hipEventQuery(r->last) != hipSuccess) continue;
        if (!victim || r->last_use < victim->last_use) victim = r;
      }
      if (!victim) return false;
      drop(victim);
      ++evictions;
    }
    return true;
  }

  void drop(Resident* r) {
    if (r->h) spike_destroy(r->h);
    if (r->bytes) pool->release(r->off, r->bytes);
    if (r->last) event_pool.push_back(r->last);
    res.erase(r->id);
    delete r;
  }

  // Resident factorisation for the request, factoring it when needed;
  // nullptr when it does not fit now (retry later).
  Resident* resident_for(Req* q, int* err) {
    *err = 0;
    auto it = res.find(q->r.matrix_id);
    if (it != res.end()) {
      const Resident* r = it->second;
      if (r->n != q->r.n || r->kl != q->r.kl || r->ku != q->r.ku || r->dAB != q->r.dAB) {
        *err = -101;   // the id is resident for another matrix
        return nullptr;
      }
      return it->second;
    }
    size_t need = 0;
    int e = spike_workspace_size(q->r.n, q->r.kl, q->r.ku, &q->r.opts, &need);
    if (e) {
      *err = e;
      return nullptr;
    }
    if (need > pool->cap()) {
      *err = -100;   // larger than the whole budget
      return nullptr;
    }
    size_t off = 0;
    if (!make_room(need, &off)) return nullptr;
    Resident* r = new Resident();
    r->id = q->r.matrix_id;
    r->n = q->r.n;
    r->kl = q->r.kl;
    r->ku = q->r.ku;
    r->dAB = q->r.dAB;
    r->off = off;
    r->bytes = need;
    r->stream = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    r->last = take_event();
    // factored with the other new matrices of this pass (flush_factors)
    r->freq = &q->r;
    deferred[r->stream].push_back(r);
    res[r->id] = r;
    return r;
  }

  // The factorisations admitted in this pass, one spike_factor_batch per
  // home stream (before the stream's solves); a resident whose factorisation
  // fails is dropped and its id's error returned through failed_ids.
  void flush_factors(std::map<int64_t, int>& failed_ids) {
    for (auto& kv : deferred) {
      std::vector<Resident*>& v = kv.second;
      if (v.empty()) continue;
      const hipStream_t st = streams[kv.first];
      const int cnt = (int)v.size();
      std::vector<int64_t> n(cnt), ld(cnt);
      std::vector<int32_t> kl(cnt), ku(cnt);
      std::vector<const double*> ab(cnt);
      std::vector<spike_opts> op(cnt);
      std::vector<void*> wk(cnt);
      std::vector<size_t> wb(cnt);
      std::vector<spike_handle> hs(cnt, nullptr);
      for (int i = 0; i < cnt; ++i) {
        const spike_request& q = *v[i]->freq;
        n[i] = q.n;
        kl[i] = q.kl;
        ku[i] = q.ku;
        ab[i] = q.dAB;
        ld[i] = q.ldab;
        op[i] = q.opts;
        wk[i] = base + v[i]->off;
        wb[i] = v[i]->bytes;
      }
      int e = spike_factor_batch(cnt, n.data(), kl.data(), ku.data(), ab.data(), ld.data(), op.data(), wk.data(),
                                 wb.data(), st, hs.data());
      for (int i = 0; i < cnt; ++i) {
        Resident* r = v[i];
        int ei = e;
        if (e) {   // find the failing system: factor the others one by one
          const spike_request& q = *r->freq;
          ei = spike_factor(q.n, q.kl, q.ku, q.dAB, q.ldab, &q.opts, base + r->off, r->bytes, st, &hs[i]);
        }
        r->freq = nullptr;
        if (ei) {
          failed_ids[r->id] = ei;
          continue;
        }
        r->h = hs[i];
        (void)hipEventRecord(r->last, st);
        ++factorizations;
      }
      v.clear();
    }
  }

  void finish(Req* q, int state, int err) {
    q->state = state;
    q->err = err;
    q->t_done = now_s();
    t_last = std::max(t_last, q->t_done);
    if (state == 2) {
      ++completed;
      lat.push_back(q->t_done - q->t_arrive);
    } else {
      ++failed;
    }
  }

  // One scheduling pass; returns true when anything changed.
  bool pass() {
    bool did = false;
    // completions
    for (size_t i = 0; i < inflight.size();) {
      Req* q = inflight[i];
      if (hipEventQuery(q->done) == hipSuccess) {
        if (!q->res->info_known) {
          spike_status ds;
          if (spike_info(q->res->h, &ds) == 0) q->res->info = ds.info;
          q->res->info_known = true;
        }
        q->info = q->res->info;
        finish(q, 2, 0);
        q->res->pending--;
        load[q->res->stream]--;
        event_pool.push_back(q->done);
        q->done = nullptr;
        inflight[i] = inflight.back();
        inflight.pop_back();
        did = true;
      } else {
        ++i;
      }
    }
    // admission, grouped into one batched solve per home stream
    std::map<int, std::vector<Req*>> batch;
    std::unordered_set<Resident*> used;
    int slots = o.max_inflight - (int)inflight.size();
    for (auto it = pending.begin(); it != pending.end() && slots > 0;) {
      Req* q = *it;
      int err = 0;
      Resident* r = resident_for(q, &err);
      if (err) {
        finish(q, 3, err);
        it = pending.erase(it);
        did = true;
        continue;
      }
      // A request waiting for pool memory stops admission behind it, so the
      // residents it needs evicted go idle and it cannot be starved.
      if (!r) break;
      if (used.count(r) || (int)batch[r->stream].size() >= o.batch_window) {
        ++it;
        continue;
      }
      used.insert(r);
      q->res = r;
      r->pending++;
      r->last_use = ++clock;
      load[r->stream]++;
      batch[r->stream].push_back(q);
      it = pending.erase(it);
      --slots;
      did = true;
    }
    std::map<int64_t, int> failed_ids;
    flush_factors(failed_ids);
    if (!failed_ids.empty()) {
      for (auto& kv : batch) {
        std::vector<Req*>& v = kv.second;
        for (size_t i = 0; i < v.size();) {
          auto f = failed_ids.find(v[i]->r.matrix_id);
          if (f == failed_ids.end()) {
            ++i;
            continue;
          }
          Req* q = v[i];
          finish(q, 3, f->second);
          load[q->res->stream]--;
          q->res = nullptr;
          v[i] = v.back();
          v.pop_back();
        }
      }
      for (auto& kv : failed_ids) {
        auto it = res.find(kv.first);
        if (it != res.end()) {
          it->second->pending = 0;
          drop(it->second);
        }
      }
    }
    for (auto& kv : batch) {
      std::vector<Req*>& v = kv.second;
      if (v.empty()) continue;
      const hipStream_t st = streams[kv.first];
      std::vector<spike_handle> hs;
      std::vector<int32_t> nr, tr;
      std::vector<double*> bp;
      std::vector<int64_t> ld;
      for (Req* q : v) {
        hs.push_back(q->res->h);
        nr.push_back(q->r.nrhs);
        bp.push_back(q->r.dB);
        ld.push_back(q->r.ldb);
        tr.push_back(q->r.trans);
      }
      const int e = spike_solve_batch(hs.data(), nr.data(), bp.data(), ld.data(), tr.data(), (int32_t)v.size(), st);
      for (Req* q : v) {
        if (e) {
          finish(q, 3, e);
          q->res->pending--;
          load[q->res->stream]--;
          continue;
        }
        q->done = take_event();
        (void)hipEventRecord(q->done, st);
        (void)hipEventRecord(q->res->last, st);
        q->state = 1;
        inflight.push_back(q);
      }
    }
    return did;
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      const bool did = pass();
      if (did) cv_done.notify_all();
      if (stop && pending.empty() && inflight.empty()) break;
      if (!did) {
        if (inflight.empty() && pending.empty()) cv_work.wait(lk);
        else cv_work.wait_for(lk, std::chrono::microseconds(20));
      }
    }
  }
};

namespace {
constexpr uint32_t kServerMagic = 0x5e7e5u;
bool valid(spike_server s) { return s && s->magic == kServerMagic; }
}  // namespace

extern "C" {

void spike_server_default_opts(spike_server_opts* o) {
  if (!o) return;
  o->hbm_budget = (size_t)16 << 30;
  o->max_inflight = 64;
  o->streams = 4;
  o->batch_window = 32;
  o->dpool = nullptr;
}

int spike_server_create(const spike_server_opts* opts, spike_server* out) {
  if (!out) return -2;
  spike_server_opts o;
  spike_server_default_opts(&o);
  if (opts) o = *opts;
  if (o.hbm_budget < 4096 || o.max_inflight < 1 || o.streams < 1 || o.streams > 16 || o.batch_window < 1 ||
      o.dpool == nullptr || (reinterpret_cast<uintptr_t>(o.dpool) & 255u) != 0)
    return -1;
  spike_server s = new (std::nothrow) spike_server_s();
  if (!s) return SPIKE_ERR_HIP - (int)hipErrorOutOfMemory;
  s->o = o;
  (void)hipGetDevice(&s->device);
  s->base = static_cast<char*>(o.dpool);
  hipError_t e = hipSuccess;
  s->pool = new Pool(o.hbm_budget);
  for (int i = 0; i < o.streams; ++i) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
    s->streams.push_back(st);
    s->load.push_back(0);
  }
  if ((int)s->streams.size() != o.streams) {
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s->pool;
    delete s;
    return SPIKE_ERR_HIP - (int)e;
  }
  s->magic = kServerMagic;
  s->worker = std::thread([s] { s->loop(); });
  *out = s;
  return 0;
}

int spike_server_submit(spike_server s, const spike_request* r, int64_t* ticket) {
  if (!valid(s)) return -1;
  if (!r || r->n < 1 || r->kl < 0 || r->ku < 0 || !r->dAB || r->ldab < (int64_t)r->kl + r->ku + 1 ||
      r->nrhs < 1 || !r->dB || r->ldb < r->n)
    return -2;
  if (!ticket) return -3;
  Req* q = new (std::nothrow) Req();
  if (!q) return SPIKE_ERR_HIP - (int)hipErrorOutOfMemory;
  q->r = *r;
  q->t_arrive = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return -1;
    }
    q->ticket = s->next_ticket++;
    if (s->reqs.empty() || s->t_first == 0) s->t_first = q->t_arrive;
    s->reqs[q->ticket] = q;
    s->pending.push_back(q);
    *ticket = q->ticket;
  }
  s->cv_work.notify_one();
  return 0;
}

static void fill_status(const Req* q, spike_request_status* st) {
  st->state = q->state;
  st->error = q->err;
  st->info = q->info;
  st->latency_s = q->state >= 2 ? q->t_done - q->t_arrive : -1.0;
}

int spike_server_poll(spike_server s, int64_t ticket, spike_request_status* st) {
  if (!valid(s)) return -1;
  if (!st) return -3;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return -2;
  fill_status(it->second, st);
  return 0;
}

int spike_server_wait(spike_server s, int64_t ticket, spike_request_status* st) {
  if (!valid(s)) return -1;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return -2;
  Req* q = it->second;
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [q] { return q->state >= 2; });
  if (st) fill_status(q, st);
  return 0;
}

int spike_server_release(spike_server s, int64_t ticket) {
  if (!valid(s)) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return -2;
  if (it->second->state < 2) return -3;   // still queued or on the device
  delete it->second;
  s->reqs.erase(it);
  return 0;
}

int spike_server_drain(spike_server s) {
  if (!valid(s)) return -1;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [s] { return s->pending.empty() && s->inflight.empty(); });
  return 0;
}

int spike_server_stats(spike_server s, spike_server_report* out) {
  if (!valid(s)) return -1;
  if (!out) return -2;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = s->completed;
  out->failed = s->failed;
  out->factorizations = s->factorizations;
  out->evictions = s->evictions;
  out->resident = (int64_t)s->res.size();
  out->hbm_used = s->pool->used();
  out->hbm_high_water = s->pool->hwm();
  std::vector<double> l = s->lat;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
      const size_t i = (size_t)std::min<double>(l.size() - 1, std::floor(q * (l.size() - 1) + 0.5));
      return l[i];
    };
    out->p50_s = pct(0.50);
    out->p99_s = pct(0.99);
    out->max_s = l.back();
    const double span = s->t_last - s->t_first;
    out->solves_per_s = span > 0 ? (double)s->completed / span : 0.0;
  }
  return 0;
}

int spike_server_destroy(spike_server s) {
  if (!valid(s)) return -1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->worker.join();
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  std::vector<Resident*> rs;
  for (auto& kv : s->res) rs.push_back(kv.second);
  for (Resident* r : rs) s->drop(r);
  for (auto& kv : s->reqs) {
    if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    delete kv.second;
  }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s->pool;
  s->magic = 0;
  delete s;
  return 0;
}

}  // extern "C"
