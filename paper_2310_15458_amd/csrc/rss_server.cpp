// Solve server of librss: keeps factorizations resident in HBM and serves
// factor and solve requests with continuous batching.
//
//  * A factor worker (its own HIP stream) admits queued factor jobs while the
//    device-memory budget allows, evicting least-recently-used factorizations
//    that no pending solve pins, and factors them one at a time.
//  * A solve worker (its own stream) repeatedly takes every pending solve
//    whose factorization is resident, up to max_batch, and runs them as one
//    batched solve (rss_solve_batch: one launch per tree level and colour over
//    all of them, refinement included).  Requests arriving meanwhile wait for
//    the next tick; factor and solve work overlap on the device.
//  * Completions carry submit / start / end times for latency statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rss.h"

namespace rss {
// defined with the host driver: marks the server's worker threads, whose
// merged solve batches reuse tuned solve tiles without tuning
extern thread_local bool g_server_thread;
}  // namespace rss

namespace {

using Clock = std::chrono::steady_clock;

struct Entry {
  rss_handle h = nullptr;
  int state = 0;          // 0 queued, 1 factoring, 2 resident, 3 evicted, 4 failed
  double bytes = 0;       // device bytes held (resident)
  double est = 0;         // admission estimate
  int pins = 0;           // pending solves
  double last_use = 0;
  int64_t n = 0;
};

struct FactorJob {
  int64_t id;
  std::vector<double> pts;
  rss_kernel k;
  double t_submit;
};

struct SolveJob {
  int64_t req, id;
  void* B;
  int nrhs;
  double t_submit;
};

}  // namespace

struct rss_server {
  rss_server_options o{};
  std::mutex mu;
  std::condition_variable cv_f, cv_s, cv_done;
  std::map<int64_t, Entry> ent;
  std::deque<FactorJob> fq;
  std::deque<SolveJob> sq;
  std::deque<rss_completion> done;
  int64_t next_id = 1;
  double used = 0;  // bytes of resident + factoring entries
  bool stop = false;
  Clock::time_point t0 = Clock::now();
  hipStream_t fs = nullptr, ss = nullptr;
  std::thread tf, ts;
  double bytes_per_unknown = 0;  // running estimate for admission
  rss_server_stats st{};

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // estimated device bytes of a factorization of n unknowns
  double estimate(int64_t n) const {
    const double per = bytes_per_unknown > 0 ? bytes_per_unknown
                                             : (o.precision == RSS_FP32_REFINE ? 60e3 : 120e3);
    return per * (double)n;
  }

  // evict least-recently-used resident entries without pins until need fits (mu held)
  bool make_room(double need) {
    while (used + need > o.budget_bytes) {
      int64_t victim = -1;
      double oldest = 1e300;
      for (auto& kv : ent)
        if (kv.second.state == 2 && kv.second.pins == 0 && kv.second.last_use < oldest) {
          oldest = kv.second.last_use;
          victim = kv.first;
        }
      if (victim < 0) return false;
      Entry& e = ent[victim];
      rss_free(e.h);
      e.h = nullptr;
      e.state = 3;
      used -= e.bytes;
      st.evictions++;
    }
    return true;
  }

  void factor_loop() {
    for (;;) {
      FactorJob job;
      double need = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop && fq.empty()) return;
          if (!fq.empty()) {
            need = estimate((int64_t)fq.front().pts.size() / 2);
            if (make_room(need)) break;
            // nothing left to evict or wait for: the estimate is only a guess, so
            // an empty server always admits the job
            if (used == 0) break;
          }
          cv_f.wait_for(lk, std::chrono::milliseconds(20));
        }
        job = std::move(fq.front());
        fq.pop_front();
        Entry& e = ent[job.id];
        e.state = 1;
        e.est = need;
        used += need;
      }
      rss_completion c{};
      c.req = job.id;
      c.kind = 0;
      c.t_submit = job.t_submit;
      c.t_start = now();
      rss_options opt{};
      opt.precision = (rss_precision)o.precision;
      opt.n_proxy = o.n_proxy;
      opt.refine_tol = o.refine_tol;
      opt.max_refine = o.max_refine;
      opt.stream = fs;
      rss_handle h = nullptr;
      const int64_t n = (int64_t)job.pts.size() / 2;
      const int rc = rss_factor_ex(job.pts.data(), n, &job.k, o.tol, o.leaf, &opt, &h);
      c.t_end = now();
      c.status = rc;
      {
        std::lock_guard<std::mutex> lk(mu);
        Entry& e = ent[job.id];
        used -= e.est;
        if (rc == RSS_OK) {
          rss_stats s{};
          rss_info(h, &s);
          rss_set_stream(h, ss);  // solves of this factorization run on the solve stream
          e.h = h;
          e.bytes = s.device_bytes;
          e.n = n;
          e.state = 2;
          e.last_use = now();
          used += e.bytes;
          const double per = e.bytes / (double)n;
          bytes_per_unknown = bytes_per_unknown > 0 ? std::max(bytes_per_unknown, per) : per;
          st.factored++;
          st.peak_bytes = std::max(st.peak_bytes, used);
        } else {
          e.state = 4;
        }
        done.push_back(c);
      }
      cv_s.notify_all();
      cv_done.notify_all();
    }
  }

  void solve_loop() {
    for (;;) {
      std::vector<SolveJob> batch;
      std::vector<rss_handle> hs;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          // ready: target resident (or failed/evicted -> completes with an error)
          for (auto it = sq.begin(); it != sq.end() && (int)batch.size() < o.max_batch;) {
            Entry& e = ent[it->id];
            if (e.state == 2) {
              batch.push_back(*it);
              hs.push_back(e.h);
              it = sq.erase(it);
            } else if (e.state >= 3) {
              rss_completion c{};
              c.req = it->req;
              c.kind = 1;
              c.status = RSS_EINVAL;
              c.t_submit = it->t_submit;
              c.t_start = c.t_end = now();
              done.push_back(c);
              e.pins--;
              it = sq.erase(it);
              cv_done.notify_all();
            } else {
              ++it;
            }
          }
          if (!batch.empty()) break;
          if (stop && sq.empty()) return;
          cv_s.wait_for(lk, std::chrono::milliseconds(5));
        }
      }
      const double ts0 = now();
      std::vector<void*> Bs;
      std::vector<int> nr;
      for (auto& j : batch) {
        Bs.push_back(j.B);
        nr.push_back(j.nrhs);
      }
      // entries of one batch share precision and refinement mode by construction
      const int rc = rss_solve_batch((int)batch.size(), hs.data(), Bs.data(), nr.data());
      const double ts1 = now();
      {
        std::lock_guard<std::mutex> lk(mu);
        st.batches++;
        st.batched_solves += (int64_t)batch.size();
        st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, (int64_t)batch.size());
        for (size_t i = 0; i < batch.size(); ++i) {
          Entry& e = ent[batch[i].id];
          rss_stats s{};
          rss_info(hs[i], &s);
          rss_completion c{};
          c.req = batch[i].req;
          c.kind = 1;
          c.status = rc;
          c.t_submit = batch[i].t_submit;
          c.t_start = ts0;
          c.t_end = ts1;
          c.relres = s.last_relres;
          c.iters = s.last_iters;
          c.batch = (int)batch.size();
          done.push_back(c);
          e.pins--;
          e.last_use = ts1;
          st.solved_unknowns += (double)e.n * batch[i].nrhs;
        }
      }
      cv_f.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

int rss_server_create(const rss_server_options* o, rss_server_t* out) {
  if (!o || !out) return RSS_EINVAL;
  *out = nullptr;
  if (!(o->budget_bytes > 0) || o->tol <= 0 || o->leaf < 1) return RSS_EINVAL;
  std::unique_ptr<rss_server> s(new rss_server());
  s->o = *o;
  if (s->o.max_batch <= 0) s->o.max_batch = 64;
  if (hipStreamCreateWithFlags(&s->fs, hipStreamNonBlocking) != hipSuccess) return RSS_EHIP;
  if (hipStreamCreateWithFlags(&s->ss, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(s->fs);
    return RSS_EHIP;
  }
  rss_server* p = s.get();
  p->tf = std::thread([p] {
    rss::g_server_thread = true;
    p->factor_loop();
  });
  p->ts = std::thread([p] {
    rss::g_server_thread = true;
    p->solve_loop();
  });
  *out = s.release();
  return RSS_OK;
}

int rss_server_factor(rss_server_t s, const double* points, int64_t n, const rss_kernel* k,
                      int64_t* id) {
  if (!s || !points || !k || !id || n < 1) return RSS_EINVAL;
  FactorJob j;
  j.pts.assign(points, points + 2 * n);
  j.k = *k;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j.id = s->next_id++;
    j.t_submit = s->now();
    Entry& e = s->ent[j.id];
    e.n = n;
    *id = j.id;
    s->fq.push_back(std::move(j));
  }
  s->cv_f.notify_all();
  return RSS_OK;
}

int rss_server_solve(rss_server_t s, int64_t id, void* B, int nrhs, int64_t* req) {
  if (!s || !B || nrhs < 1 || !req) return RSS_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->ent.find(id);
    if (it == s->ent.end() || it->second.state >= 3) return RSS_EINVAL;
    it->second.pins++;  // the factorization stays resident until this solve completes
    SolveJob j{s->next_id++, id, B, nrhs, s->now()};
    *req = j.req;
    s->sq.push_back(j);
  }
  s->cv_s.notify_all();
  return RSS_OK;
}

int rss_server_poll(rss_server_t s, rss_completion* out, int cap, int wait_ms, int* count) {
  if (!s || !out || !count || cap < 1) return RSS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty(); });
  int c = 0;
  while (c < cap && !s->done.empty()) {
    out[c++] = s->done.front();
    s->done.pop_front();
  }
  *count = c;
  return RSS_OK;
}

int rss_server_stats_get(rss_server_t s, rss_server_stats* out) {
  if (!s || !out) return RSS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->used_bytes = s->used;
  int64_t res = 0;
  for (auto& kv : s->ent) res += kv.second.state == 2;
  out->resident = res;
  out->pending = (int64_t)(s->fq.size() + s->sq.size());
  return RSS_OK;
}

int rss_server_destroy(rss_server_t s) {
  if (!s) return RSS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_f.notify_all();
  s->cv_s.notify_all();
  if (s->tf.joinable()) s->tf.join();
  if (s->ts.joinable()) s->ts.join();
  for (auto& kv : s->ent)
    if (kv.second.h) rss_free(kv.second.h);
  (void)hipStreamDestroy(s->fs);
  (void)hipStreamDestroy(s->ss);
  delete s;
  return RSS_OK;
}

}  // extern "C"
