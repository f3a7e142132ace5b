// Solve server of librss: keeps factorizations resident in HBM and serves
// factor and solve requests with continuous batching.
//
//  * A factor worker (its own HIP stream) admits queued factor jobs while the
//    device-memory budget allows, evicting least-recently-used factorizations
//    that no pending solve pins, and factors them one at a time.
//  * A solve worker (its own stream) keeps a set of solves in flight and
//    advances all of them by one refinement step at a time: one batched
//    application of the factored inverses over all of them (one launch per
//    tree level and colour, Sec. 2.6), then their residuals.  Before every
//    step it admits pending solves whose factorization is resident (up to
//    max_batch in flight), and after it retires every solve that converged,
//    so a solve arriving mid-refinement joins at the next step instead of
//    waiting for the others to finish.  Factor and solve work overlap on the
//    device (two streams).
//  * With grid_residual, a factorization whose points form a uniform grid of
//    cell centres gets an FFT product (rss_gridop_*) as its refinement
//    residual; its memory counts towards the budget.
//  * Completions carry submit / start / end times for latency statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rss.h"

struct rss_ctx;
namespace rss {
// defined with the host driver: marks the server's worker threads, whose
// merged solve batches reuse tuned solve tiles without tuning
extern thread_local bool g_server_thread;
// refined solves one step at a time (host driver)
int refine_begin(::rss_ctx* h, void* B, int nrhs, void** job);
int refine_step(void* const* jobs, int n);
bool refine_done(const void* job);
int refine_finish(void* job, double* relres, int* iters);
void refine_free(void* job);
}  // namespace rss

namespace {

using Clock = std::chrono::steady_clock;

struct Entry {
  rss_handle h = nullptr;
  rss_gridop_t gop = nullptr;  // FFT residual of a grid problem (grid_residual)
  int state = 0;          // 0 queued, 1 factoring, 2 resident, 3 evicted, 4 failed
  double bytes = 0;       // device bytes held (resident)
  double est = 0;         // admission estimate
  int pins = 0;           // pending solves
  double last_use = 0;
  int64_t n = 0;
  // the problem, kept on the host so that an evicted factorization can be redone
  std::shared_ptr<const std::vector<double>> pts;
  rss_kernel k{};
};

struct FactorJob {
  int64_t id;
  std::shared_ptr<const std::vector<double>> pts;
  rss_kernel k;
  double t_submit;
  bool redo;  // refactoring an evicted entry for a solve: no completion is reported
};

struct SolveJob {
  int64_t req, id;
  void* B;
  int nrhs;
  double t_submit;
};

// a solve in flight: its refinement job and admission time
struct Flight {
  SolveJob j;
  void* job;
  double t_start;
  double bytes;  // working bytes
};

// the points are the cell centres of an n x n grid, point index iy n + ix
bool as_grid(const std::vector<double>& pts, int& n, double& x0, double& y0, double& h) {
  const int64_t N = (int64_t)pts.size() / 2;
  n = (int)std::llround(std::sqrt((double)N));
  if (n < 2 || (int64_t)n * n != N || n > 2048) return false;
  h = pts[2] - pts[0];
  if (!(h > 0)) return false;
  x0 = pts[0] - 0.5 * h;
  y0 = pts[1] - 0.5 * h;
  for (int64_t i = 0; i < N; ++i) {
    const double gx = x0 + ((double)(i % n) + 0.5) * h, gy = y0 + ((double)(i / n) + 0.5) * h;
    if (std::fabs(pts[2 * i] - gx) > 1e-9 * h || std::fabs(pts[2 * i + 1] - gy) > 1e-9 * h) return false;
  }
  return true;
}

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
  double inflight = 0;  // working bytes of the solves in flight
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

  double factor_budget() const { return 0.75 * o.budget_bytes; }
  double solve_budget() const { return 0.25 * o.budget_bytes; }
  // device working bytes of a solve (right-hand sides, iterate, residual, best
  // iterate, and the FP32 correction)
  double solve_bytes(int64_t n, int nrhs) const {
    return (double)n * nrhs * (o.precision == RSS_FP32_REFINE ? 72.0 : 64.0);
  }

  // evict least-recently-used resident entries without pins until need fits (mu held)
  bool make_room(double need) {
    while (used + need > factor_budget()) {
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
      rss_gridop_free(e.gop);
      e.gop = nullptr;
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
            need = estimate((int64_t)fq.front().pts->size() / 2);
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
      const int64_t n = (int64_t)job.pts->size() / 2;
      const int rc = rss_factor_ex(job.pts->data(), n, &job.k, o.tol, o.leaf, &opt, &h);
      rss_gridop_t gop = nullptr;
      double gop_bytes = 0;
      int gn = 0;
      double gx0 = 0, gy0 = 0, gh = 0;
      if (rc == RSS_OK && o.grid_residual && job.k.kind != RSS_DEGENERATE &&
          as_grid(*job.pts, gn, gx0, gy0, gh) &&
          rss_gridop_create(&job.k, gn, gx0, gy0, gh, fs, &gop) == RSS_OK) {
        rss_set_residual_op(h, gop);
        const double M = (double)(1 << (int)std::ceil(std::log2(2.0 * gn - 1.0)));
        // generator transform, point data and a 16-column work array
        gop_bytes = M * M * 16 + (double)gn * gn * 24 + 16.0 * gn * M * 16;
      }
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
          e.gop = gop;
          e.bytes = s.device_bytes + gop_bytes;
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
          std::fprintf(stderr, "rss_server: factor job %lld failed: %s (%s)\n", (long long)job.id,
                       rss_error_string(rc), rss_last_error());
        }
        if (!job.redo) done.push_back(c);
      }
      cv_s.notify_all();
      cv_done.notify_all();
    }
  }

  void complete_solve(const Flight& f, int status, double relres, int iters, int width, double t_end) {
    // mu held
    Entry& e = ent[f.j.id];
    rss_completion c{};
    c.req = f.j.req;
    c.kind = 1;
    c.status = status;
    c.t_submit = f.j.t_submit;
    c.t_start = f.t_start;
    c.t_end = t_end;
    c.relres = relres;
    c.iters = iters;
    c.batch = width;
    done.push_back(c);
    e.pins--;
    e.last_use = t_end;
    inflight -= f.bytes;
    st.solved_unknowns += (double)e.n * f.j.nrhs;
  }

  void solve_loop() {
    std::vector<Flight> fl;
    for (;;) {
      std::vector<SolveJob> admit;
      std::vector<double> admit_bytes;
      std::vector<rss_handle> admit_h;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          // admit: target resident (or failed/evicted -> completes with an error)
          for (auto it = sq.begin(); it != sq.end() && (int)(fl.size() + admit.size()) < o.max_batch;) {
            Entry& e = ent[it->id];
            if (e.state == 2) {
              // first come, first admitted: a solve whose buffers do not fit
              // waits, and so does everything behind it
              const double b = solve_bytes(e.n, it->nrhs);
              if (inflight + b > solve_budget() && !(fl.empty() && admit.empty())) break;
              inflight += b;
              st.inflight_peak_bytes = std::max(st.inflight_peak_bytes, inflight);
              admit.push_back(*it);
              admit_bytes.push_back(b);
              admit_h.push_back(e.h);
              it = sq.erase(it);
            } else if (e.state == 4) {  // its factorization failed
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
          if (!fl.empty() || !admit.empty()) break;
          if (stop && sq.empty()) return;
          cv_s.wait_for(lk, std::chrono::milliseconds(5));
        }
      }
      const double t_adm = now();
      for (size_t i = 0; i < admit.size(); ++i) {
        void* job = nullptr;
        const int rc = rss::refine_begin(admit_h[i], admit[i].B, admit[i].nrhs, &job);
        if (rc == RSS_OK) {
          fl.push_back({admit[i], job, t_adm, admit_bytes[i]});
        } else {
          std::lock_guard<std::mutex> lk(mu);
          complete_solve({admit[i], nullptr, t_adm, admit_bytes[i]}, rc, -1.0, 0, 0, now());
          cv_done.notify_all();
        }
      }
      if (fl.empty()) continue;
      // one step of every solve in flight
      std::vector<void*> jobs;
      for (auto& f : fl) jobs.push_back(f.job);
      const int rc = rss::refine_step(jobs.data(), (int)jobs.size());
      const int width = (int)fl.size();
      std::vector<Flight> keep;
      std::vector<std::pair<Flight, std::pair<int, std::pair<double, int>>>> fin;
      for (auto& f : fl) {
        if (rc != RSS_OK) {
          rss::refine_free(f.job);
          fin.push_back({f, {rc, {-1.0, 0}}});
        } else if (rss::refine_done(f.job)) {
          double rr = -1.0;
          int it = 0;
          const int code = rss::refine_finish(f.job, &rr, &it);
          fin.push_back({f, {code, {rr, it}}});
        } else {
          keep.push_back(f);
        }
      }
      fl.swap(keep);
      {
        std::lock_guard<std::mutex> lk(mu);
        st.batches++;
        st.batched_solves += width;
        st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, width);
        const double t_end = now();
        for (auto& x : fin) complete_solve(x.first, x.second.first, x.second.second.first,
                                           x.second.second.second, width, t_end);
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
  j.pts = std::make_shared<const std::vector<double>>(points, points + 2 * n);
  j.k = *k;
  j.redo = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j.id = s->next_id++;
    j.t_submit = s->now();
    Entry& e = s->ent[j.id];
    e.n = n;
    e.pts = j.pts;
    e.k = j.k;
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
    if (it == s->ent.end() || it->second.state == 4) return RSS_EINVAL;
    Entry& e = it->second;
    if (e.state == 3) {
      // evicted: factor it again (queued behind the factor jobs already waiting)
      e.state = 0;
      s->fq.push_back(FactorJob{id, e.pts, e.k, s->now(), true});
      s->st.refactors++;
      s->cv_f.notify_all();
    }
    e.pins++;  // the factorization stays resident until this solve completes
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
  out->inflight_bytes = s->inflight;
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
  for (auto& kv : s->ent) {
    if (kv.second.h) rss_free(kv.second.h);
    rss_gridop_free(kv.second.gop);
  }
  (void)hipStreamDestroy(s->fs);
  (void)hipStreamDestroy(s->ss);
  delete s;
  return RSS_OK;
}

}  // extern "C"
