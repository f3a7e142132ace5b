// Host-logic driver: exercises the planner, batched factor/apply/solve and the
// server (admission, eviction, batching) with the kernels stubbed out.
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "rss.h"

static std::vector<double> grid(int n) {
  std::vector<double> p(2 * n * n);
  for (int iy = 0; iy < n; ++iy)
    for (int ix = 0; ix < n; ++ix) {
      p[2 * (iy * n + ix)] = (ix + 0.5) / n;
      p[2 * (iy * n + ix) + 1] = (iy + 0.5) / n;
    }
  return p;
}

#define CHECK(x)                                                   \
  do {                                                             \
    int rc_ = (x);                                                 \
    if (rc_ != RSS_OK && rc_ != RSS_ENOCONV) {                     \
      printf("FAIL %s -> %d (%s)\n", #x, rc_, rss_last_error());   \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main() {
  // single problem, both precisions, both schedules
  for (int run = 0; run < 4; ++run) {
    const int prec = run & 1;
    auto P = grid(48);
    rss_kernel k{RSS_HELMHOLTZ2D, 30.0, 1.0 / (48 * 48), 1.0, 2};
    rss_options o{};
    o.precision = (rss_precision)prec;
    o.colours = run < 2 ? 9 : 4;
    rss_handle h;
    CHECK(rss_factor_ex(P.data(), 48 * 48, &k, 1e-6, 36, &o, &h));
    std::vector<double> B(2 * 48 * 48 * 3);
    CHECK(rss_solve(h, B.data(), 3));
    CHECK(rss_apply(h, B.data(), 3));
    rss_free(h);
  }
  // a batch with different depths, including a tree too shallow to compress
  {
    const int sides[5] = {16, 24, 32, 4, 40};
    std::vector<std::vector<double>> pts;
    std::vector<const double*> pp;
    std::vector<int64_t> n;
    std::vector<rss_kernel> ks;
    for (int i = 0; i < 5; ++i) {
      pts.push_back(grid(sides[i]));
      n.push_back((int64_t)sides[i] * sides[i]);
      ks.push_back(rss_kernel{i % 2 ? RSS_LAPLACE2D : RSS_HELMHOLTZ2D, 10.0 + i,
                              1.0 / n.back(), 1.0, 2});
    }
    for (auto& v : pts) pp.push_back(v.data());
    rss_handle hs[5];
    CHECK(rss_factor_batch(5, pp.data(), n.data(), ks.data(), 1e-6, 9, nullptr, hs));
    std::vector<std::vector<double>> Bs;
    std::vector<void*> bp;
    std::vector<int> nr;
    for (int i = 0; i < 5; ++i) {
      Bs.emplace_back(2 * n[i] * 2);
      bp.push_back(Bs.back().data());
      nr.push_back(2);
    }
    CHECK(rss_apply_batch(5, hs, bp.data(), nr.data()));
    CHECK(rss_solve_batch(5, hs, bp.data(), nr.data()));
    for (int i = 4; i >= 0; --i) rss_free(hs[i]);
  }
  // the server: a budget that forces evictions, solves pinned to their factorizations
  {
    rss_server_options o{};
    o.budget_bytes = 3e6;
    o.precision = RSS_FP32_REFINE;
    o.tol = 1e-6;
    o.leaf = 64;
    o.max_refine = 2;
    rss_server_t s;
    CHECK(rss_server_create(&o, &s));
    std::vector<std::vector<double>> bufs;
    std::vector<int64_t> ids;
    int expect = 0;
    for (int j = 0; j < 10; ++j) {
      const int n = (j % 2) ? 48 : 32;
      auto P = grid(n);
      rss_kernel k{RSS_HELMHOLTZ2D, 20.0 + j, 1.0 / (n * n), 1.0, 2};
      int64_t id;
      CHECK(rss_server_factor(s, P.data(), (int64_t)n * n, &k, &id));
      ids.push_back(id);
      ++expect;
      for (int q = 0; q < 3; ++q) {
        bufs.emplace_back(2 * n * n * 4);
        int64_t req;
        CHECK(rss_server_solve(s, id, bufs.back().data(), 4, &req));
        ++expect;
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
    int got = 0, bad = 0;
    rss_completion c[64];
    int cnt;
    for (int spins = 0; got < expect && spins < 600; ++spins) {
      CHECK(rss_server_poll(s, c, 64, 50, &cnt));
      got += cnt;
      for (int i = 0; i < cnt; ++i) bad += (c[i].status != RSS_OK && c[i].status != RSS_ENOCONV);
    }
    rss_server_stats st;
    CHECK(rss_server_stats_get(s, &st));
    printf("server: completions %d/%d failed %d factored %ld evictions %ld batches %ld max_batch %ld\n",
           got, expect, bad, (long)st.factored, (long)st.evictions, (long)st.batches,
           (long)st.max_batch_seen);
    CHECK(rss_server_destroy(s));
    if (got != expect || bad || st.factored != 10 || st.evictions < 1) {
      printf("FAIL server\n");
      return 1;
    }
  }
  printf("OK\n");
  return 0;
}
