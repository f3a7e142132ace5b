// Host driver of librss: the C ABI (include/rss.h), the quadtree planner
// (Sec. 2.1), the bottom-up factorization schedule (Alg. a:fact with the
// colour ordering), the level transition (Sec. 2.5), the root, the solve
// sweeps (Sec. 2.6) and FP64 iterative refinement.
//
// Schedule: for depth d = D .. 2, for colour c = 0 .. 8 (colour of box (bx, by)
// is (bx mod 3) + 3 (by mod 3)), the boxes of colour c are eliminated together.
// Same-colour boxes are at least 3 boxes apart, so by Rem. r:t and Rem. r:nn
// they touch disjoint blocks and the result equals the sequential order
// "colour-major, ascending id within a colour".  Sizes that the ranks decide
// stay on the device within a depth; the host reads them back once per depth
// to lay out the next one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rss.h"
#include "rss_internal.h"

using namespace rss;

namespace {

thread_local std::string g_err;

struct Fail {
  int code;
};

void fail(int code, const std::string& msg) {
  g_err = msg;
  throw Fail{code};
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      fail(RSS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                     \
  } while (0)

constexpr int MAX_DEPTH = 15;
constexpr int MIN_DEPTH = 2;  // compressed depths are D .. 2 (4 x 4 boxes and finer)

// device memory owned by a handle
struct Arena {
  std::vector<void*> ptrs;
  double bytes = 0;
  void* alloc(size_t n) {
    if (n == 0) n = 16;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(RSS_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    ptrs.push_back(p);
    bytes += (double)n;
    return p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      (void)hipFree(p);
      ptrs.erase(it);
    }
  }
  ~Arena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* up(const std::vector<T>& v, hipStream_t s) {
    T* p = (T*)alloc(v.size() * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
};

int chebyshev(int nb, int a, int b) {
  return std::max(std::abs(a % nb - b % nb), std::abs(a / nb - b / nb));
}

// 8 neighbours / 16 distance-2 boxes, ascending id, clipped to the grid
std::vector<int> ring(int nb, int b, int r) {
  std::vector<int> out;
  const int bx = b % nb, by = b / nb;
  for (int y = by - r; y <= by + r; ++y)
    for (int x = bx - r; x <= bx + r; ++x)
      if (x >= 0 && y >= 0 && x < nb && y < nb && std::max(std::abs(x - bx), std::abs(y - by)) == r)
        out.push_back(y * nb + x);
  return out;
}

struct LevelHost {
  int d = 0, nb = 0;
  std::vector<int> n0;
  std::vector<int64_t> ioff, boff;
  std::vector<int> idx;  // initial active ids (ascending per box)
  int64_t nA = 0;
  int nmax = 0, mmax = 0, nNmax = 0, msum_max = 0;
  // device
  int* d_n0 = nullptr;
  int* d_cur = nullptr;
  int* d_idx = nullptr;
  int64_t* d_ioff = nullptr;
  int64_t* d_boff = nullptr;
  void* d_A = nullptr;

  void layout(int depth, const std::vector<int>& counts) {
    d = depth;
    nb = 1 << d;
    const int nbox = nb * nb;
    n0 = counts;
    ioff.assign(nbox, 0);
    int64_t o = 0;
    for (int b = 0; b < nbox; ++b) {
      ioff[b] = o;
      o += n0[b];
      nmax = std::max(nmax, n0[b]);
    }
    boff.assign((size_t)nbox * 25, -1);
    int64_t a = 0;
    for (int b = 0; b < nbox; ++b) {
      const int bx = b % nb, by = b / nb;
      int nsum = 0, msum = 0;
      for (int s = 0; s < 25; ++s) {
        const int x = bx + s % 5 - 2, y = by + s / 5 - 2;
        if (x < 0 || y < 0 || x >= nb || y >= nb) continue;
        const int b2 = y * nb + x;
        boff[(size_t)b * 25 + s] = a;
        a += (int64_t)n0[b] * n0[b2];
        const int dd = std::max(std::abs(s % 5 - 2), std::abs(s / 5 - 2));
        if (dd == 1) nsum += n0[b2];
        if (dd == 2) msum += n0[b2];
      }
      nNmax = std::max(nNmax, nsum);
      msum_max = std::max(msum_max, msum);
    }
    nA = a;
  }
};

struct PhaseHost {
  std::vector<int> boxes;
  int64_t C_total = 0, X_total = 0, Z_total = 0, I_total = 0;
  std::vector<int64_t> oC, oX, oZ, oI;
  int* d_box = nullptr;
  int64_t *d_oC = nullptr, *d_oX = nullptr, *d_oZ = nullptr, *d_oI = nullptr;
};

// HIP-event timing of kernel classes on the handle's stream (rss_options.profile)
struct Prof {
  bool on = false;
  struct Pair {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Pair> pairs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  template <class F>
  void run(int cls, hipStream_t s, F&& f) {
    if (!on) {
      f();
      return;
    }
    Pair p{cls, get(), get()};
    HIPCHK(hipEventRecord(p.a, s));
    f();
    HIPCHK(hipEventRecord(p.b, s));
    pairs.push_back(p);
  }
  // after the stream has drained: add the elapsed times into t / n
  void collect(double* t, int64_t* n) {
    for (auto& p : pairs) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      t[p.cls] += ms;
      n[p.cls] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pairs.clear();
  }
  ~Prof() {
    for (auto& p : pairs) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct DepthRecords {
  int d = 0, nb = 0;
  int kmax = 0, rmax = 0, snmax = 0;
  int* d_k = nullptr;
  int* d_r = nullptr;
  int* d_nN = nullptr;
  int64_t *d_oT = nullptr, *d_oXi = nullptr, *d_oXSNR = nullptr, *d_oY = nullptr;
  int64_t *d_oS = nullptr, *d_oR = nullptr, *d_oN = nullptr;
  void* d_F = nullptr;
  int* d_G = nullptr;
  PhaseHost ph[9];
  // host copies after the depth completes
  std::vector<int> k, r, nN, n0, m;
};

}  // namespace

struct rss_ctx {
  int64_t N = 0;
  rss_kernel kern{};
  KParams kp{};
  double tol = 0;
  int leaf = 0;
  rss_options opt{};
  int precision = RSS_FP64;
  int refine_steps = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double x0 = 0, y0 = 0, s0 = 1;
  int D = 0;
  Arena arena;
  double* d_P = nullptr;
  std::vector<DepthRecords> recs;  // index 0 .. : depths D, D-1, ..., 2
  int n_root = 0;
  int* d_root_ids = nullptr;
  void* d_root_inv = nullptr;
  void* d_gemm_desc = nullptr;  // one descriptor for the root apply
  std::vector<int64_t> skel_counts_off;
  std::vector<std::vector<int>> skel_k;          // per compressed depth: k per box (-1 empty)
  std::vector<std::vector<int64_t>> skel_ids;    // per compressed depth: concatenated ids
  rss_stats stats{};
  Prof prof;
  int* d_err = nullptr;
  // solve workspaces (grown on demand)
  void* ws_root = nullptr;
  size_t ws_root_bytes = 0;
};

namespace {

KParams to_kp(const rss_kernel& k) {
  KParams p;
  p.kind = (int)k.kind;
  p.q = k.q;
  p.kappa = k.kappa;
  p.weight = k.weight;
  p.diag = k.diag;
  return p;
}

void validate(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf) {
  if (!points || !k) fail(RSS_EINVAL, "null pointer argument");
  if (n < 1) fail(RSS_EINVAL, "n must be >= 1");
  if (n > 2147483647LL) fail(RSS_EUNSUPPORTED, "more than 2^31-1 points");
  if (!(tol > 0) || !std::isfinite(tol)) fail(RSS_EINVAL, "tol must be positive and finite");
  if (leaf < 1) fail(RSS_EINVAL, "leaf must be >= 1");
  if (k->kind != RSS_LAPLACE2D && k->kind != RSS_HELMHOLTZ2D && k->kind != RSS_DEGENERATE)
    fail(RSS_EINVAL, "unknown kernel kind");
  if (k->kind == RSS_HELMHOLTZ2D && !(k->kappa > 0)) fail(RSS_EINVAL, "kappa must be > 0");
  if (k->kind == RSS_DEGENERATE && (k->q < 0 || k->q > 16)) fail(RSS_EINVAL, "q out of range");
  if (!std::isfinite(k->weight) || !std::isfinite(k->diag)) fail(RSS_EINVAL, "non-finite weight/diag");
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(points[i])) fail(RSS_EINVAL, "non-finite point coordinate");
}

void box_of(const double* P, int64_t n, double x0, double y0, double s0, int d, std::vector<int>& out) {
  const int nb = 1 << d;
  const double s = s0 / (double)nb;
  out.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    long bx = (long)std::floor((P[2 * i] - x0) / s);
    long by = (long)std::floor((P[2 * i + 1] - y0) / s);
    bx = std::min<long>(std::max<long>(bx, 0), nb - 1);
    by = std::min<long>(std::max<long>(by, 0), nb - 1);
    out[i] = (int)(by * nb + bx);
  }
}

template <class R>
Level<R> dev_level(const LevelHost& h, double x0, double y0, double s0) {
  Level<R> L;
  L.d = h.d;
  L.nb = h.nb;
  L.n0 = h.d_n0;
  L.cur = h.d_cur;
  L.idx = h.d_idx;
  L.ioff = h.d_ioff;
  L.boff = h.d_boff;
  L.A = (cx<R>*)h.d_A;
  L.x0 = x0;
  L.y0 = y0;
  L.side = s0 / (double)h.nb;
  return L;
}

template <class R>
Records<R> dev_records(const DepthRecords& d) {
  Records<R> r;
  r.k = d.d_k;
  r.r = d.d_r;
  r.nN = d.d_nN;
  r.oT = d.d_oT;
  r.oXi = d.d_oXi;
  r.oXSNR = d.d_oXSNR;
  r.oY = d.d_oY;
  r.oS = d.d_oS;
  r.oR = d.d_oR;
  r.oN = d.d_oN;
  r.F = (cx<R>*)d.d_F;
  r.G = d.d_G;
  return r;
}

template <class R>
Phase<R> dev_phase(const PhaseHost& p, void* W, int* Wi, int* mrow, int npx, double crad) {
  Phase<R> ph;
  ph.nbox = (int)p.boxes.size();
  ph.box = p.d_box;
  ph.oC = p.d_oC;
  ph.oX = p.d_oX;
  ph.oZ = p.d_oZ;
  ph.oI = p.d_oI;
  ph.mrow = mrow;
  ph.W = (cx<R>*)W;
  ph.Wi = Wi;
  ph.n_proxy = npx;
  ph.proxy_radius = crad;
  return ph;
}

void alloc_level(rss_ctx* h, LevelHost& L, size_t elem) {
  hipStream_t s = h->stream;
  L.d_n0 = h->arena.up(L.n0, s);
  L.d_cur = h->arena.up(L.n0, s);
  L.d_idx = h->arena.up(L.idx, s);
  L.d_ioff = h->arena.up(L.ioff, s);
  L.d_boff = h->arena.up(L.boff, s);
  L.d_A = h->arena.alloc((size_t)L.nA * elem);
}

void free_level(rss_ctx* h, LevelHost& L) {
  h->arena.release(L.d_n0);
  h->arena.release(L.d_cur);
  h->arena.release(L.d_idx);
  h->arena.release(L.d_ioff);
  h->arena.release(L.d_boff);
  h->arena.release(L.d_A);
  L.d_n0 = L.d_cur = L.d_idx = nullptr;
  L.d_ioff = L.d_boff = nullptr;
  L.d_A = nullptr;
}

template <class R>
void factor_impl(rss_ctx* h, const double* points) {
  hipStream_t s = h->stream;
  const int64_t N = h->N;
  const KParams kp = h->kp;
  const int npx = h->opt.n_proxy;
  const double crad = h->opt.proxy_radius;
  const size_t E = sizeof(cx<R>);

  // tree depth (Sec. 2.1)
  std::vector<int> bo;
  int D = 0;
  for (;; ++D) {
    if (D > MAX_DEPTH) fail(RSS_EUNSUPPORTED, "tree deeper than 15 levels");
    box_of(points, N, h->x0, h->y0, h->s0, D, bo);
    std::vector<int> cnt((size_t)1 << (2 * D), 0);
    int mx = 0;
    for (int64_t i = 0; i < N; ++i) mx = std::max(mx, ++cnt[bo[i]]);
    if (mx <= h->leaf) break;
  }
  h->D = D;
  h->stats.depth = D;

  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, s));

  std::vector<int> root_ids;
  std::vector<ListEntry> root_list;
  LevelHost cur;
  double flops_id = 0, flops_lu = 0, flops_y = 0, flops_schur = 0, fbytes = 0, kevals = 0;

  if (D >= MIN_DEPTH) {
    // leaf level: members sorted by global id
    {
      const int nbox = 1 << (2 * D);
      std::vector<int> counts(nbox, 0);
      for (int64_t i = 0; i < N; ++i) counts[bo[i]]++;
      cur.layout(D, counts);
      cur.idx.assign(N, 0);
      std::vector<int64_t> fillp(cur.ioff);
      for (int64_t i = 0; i < N; ++i) cur.idx[fillp[bo[i]]++] = (int)i;
      alloc_level(h, cur, E);
      Level<R> L = dev_level<R>(cur, h->x0, h->y0, h->s0);
      h->prof.run(RSS_K_ASSEMBLE, s, [&] { launch_leaf_assemble<R>(L, kp, h->d_P, s); });
      kevals += (double)cur.nA;
    }
    for (int d = D;; --d) {
      const int nb = 1 << d, nbox = nb * nb;
      DepthRecords dr;
      dr.d = d;
      dr.nb = nb;
      // worst-case record slots
      std::vector<int64_t> oT(nbox), oXi(nbox), oXSNR(nbox), oY(nbox), oS(nbox), oR(nbox), oN(nbox);
      int64_t F = 0, G = 0;
      for (int b = 0; b < nbox; ++b) {
        const int n = cur.n0[b];
        int nN0 = 0;
        for (int x : ring(nb, b, 1)) nN0 += cur.n0[x];
        const int64_t t = (int64_t)n * n;
        oT[b] = F;
        F += (t + 3) / 4 + n;
        oXi[b] = F;
        F += t;
        oXSNR[b] = F;
        F += (int64_t)(n + nN0) * n;
        oY[b] = F;
        F += (int64_t)(n + nN0) * n;
        oS[b] = G;
        G += n;
        oR[b] = G;
        G += n;
        oN[b] = G;
        G += nN0;
        dr.snmax = std::max(dr.snmax, n + nN0);
      }
      dr.kmax = dr.rmax = cur.nmax;
      dr.d_k = (int*)h->arena.alloc(nbox * sizeof(int));
      dr.d_r = (int*)h->arena.alloc(nbox * sizeof(int));
      dr.d_nN = (int*)h->arena.alloc(nbox * sizeof(int));
      HIPCHK(hipMemsetAsync(dr.d_k, 0, nbox * sizeof(int), s));
      HIPCHK(hipMemsetAsync(dr.d_r, 0, nbox * sizeof(int), s));
      HIPCHK(hipMemsetAsync(dr.d_nN, 0, nbox * sizeof(int), s));
      dr.d_oT = h->arena.up(oT, s);
      dr.d_oXi = h->arena.up(oXi, s);
      dr.d_oXSNR = h->arena.up(oXSNR, s);
      dr.d_oY = h->arena.up(oY, s);
      dr.d_oS = h->arena.up(oS, s);
      dr.d_oR = h->arena.up(oR, s);
      dr.d_oN = h->arena.up(oN, s);
      dr.d_F = h->arena.alloc((size_t)F * E);
      dr.d_G = (int*)h->arena.alloc((size_t)G * sizeof(int));

      // phases: colour-major, ascending id; per-slot workspace
      int64_t Cmax = 0, Xmax = 0, Zmax = 0, Imax = 0;
      int mmax = 0;
      for (int c = 0; c < 9; ++c) {
        PhaseHost& P = dr.ph[c];
        for (int b = 0; b < nbox; ++b) {
          if ((b % nb) % 3 + 3 * ((b / nb) % 3) != c || cur.n0[b] == 0) continue;
          const int n = cur.n0[b];
          int msum = 0, nN0 = 0;
          for (int x : ring(nb, b, 2)) msum += cur.n0[x];
          for (int x : ring(nb, b, 1)) nN0 += cur.n0[x];
          const int m = 2 * msum + 2 * npx;
          mmax = std::max(mmax, m);
          P.boxes.push_back(b);
          P.oC.push_back(P.C_total);
          P.C_total += (int64_t)m * n;
          P.oX.push_back(P.X_total);
          P.X_total += (int64_t)n * n;
          P.oZ.push_back(P.Z_total);
          P.Z_total += (int64_t)n * (n + nN0);
          P.oI.push_back(P.I_total);
          P.I_total += 3 * n;
        }
        // C, X and Z share one workspace per slot region
        for (size_t i = 0; i < P.boxes.size(); ++i) {
          P.oX[i] += P.C_total;
          P.oZ[i] += P.C_total + P.X_total;
        }
        Cmax = std::max(Cmax, P.C_total + P.X_total + P.Z_total);
        Imax = std::max(Imax, P.I_total);
        (void)Xmax;
        (void)Zmax;
        P.d_box = h->arena.up(P.boxes, s);
        P.d_oC = h->arena.up(P.oC, s);
        P.d_oX = h->arena.up(P.oX, s);
        P.d_oZ = h->arena.up(P.oZ, s);
        P.d_oI = h->arena.up(P.oI, s);
      }
      void* W = h->arena.alloc((size_t)Cmax * E);
      int* Wi = (int*)h->arena.alloc((size_t)Imax * sizeof(int));
      int* mrow = (int*)h->arena.alloc(nbox * sizeof(int));
      HIPCHK(hipMemsetAsync(mrow, 0, nbox * sizeof(int), s));
      int maxph = 0;
      for (int c = 0; c < 9; ++c) maxph = std::max(maxph, (int)dr.ph[c].boxes.size());
      GemmDesc<R>* desc = (GemmDesc<R>*)h->arena.alloc((size_t)std::max(1, maxph) * 81 * sizeof(GemmDesc<R>));

      Level<R> L = dev_level<R>(cur, h->x0, h->y0, h->s0);
      Records<R> rec = dev_records<R>(dr);
      const int chunks = (mmax + 63) / 64;
      for (int c = 0; c < 9; ++c) {
        Phase<R> ph = dev_phase<R>(dr.ph[c], W, Wi, mrow, npx, crad);
        if (ph.nbox == 0) continue;
        h->prof.run(RSS_K_BUILD_C, s, [&] { launch_build_C<R>(L, ph, kp, h->d_P, chunks, s); });
        h->prof.run(RSS_K_ID, s, [&] { launch_cpqr<R>(L, ph, rec, h->tol, cur.nmax, mmax, s); });
        h->prof.run(RSS_K_SPARSIFY, s, [&] { launch_sparsify<R>(L, ph, rec, s); });
        h->prof.run(RSS_K_INVERSE, s, [&] { launch_inverse<R>(ph, rec, h->d_err, cur.nmax, s); });
        launch_plan_y<R>(ph, rec, desc, s);
        h->prof.run(RSS_K_GEMM_Y, s, [&] { launch_gemm<R>(desc, ph.nbox, cur.nmax, cur.nmax + cur.nNmax, s); });
        h->prof.run(RSS_K_COMPACT, s, [&] { launch_compact<R>(L, ph, rec, s); });
        launch_plan_schur<R>(L, ph, rec, desc, s);
        h->prof.run(RSS_K_SCHUR, s, [&] { launch_gemm<R>(desc, ph.nbox * 81, cur.nmax, cur.nmax, s); });
      }
      HIPCHK(hipGetLastError());
      // read back the ranks and the surviving ids of this depth
      dr.k.resize(nbox);
      dr.r.resize(nbox);
      dr.nN.resize(nbox);
      dr.m.resize(nbox);
      std::vector<int> curk(nbox), ids(cur.idx.size());
      HIPCHK(hipMemcpyAsync(dr.k.data(), dr.d_k, nbox * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(dr.r.data(), dr.d_r, nbox * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(dr.nN.data(), dr.d_nN, nbox * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(dr.m.data(), mrow, nbox * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(curk.data(), cur.d_cur, nbox * sizeof(int), hipMemcpyDeviceToHost, s));
      if (!ids.empty())
        HIPCHK(hipMemcpyAsync(ids.data(), cur.d_idx, ids.size() * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      h->prof.collect(h->stats.t_class_ms, h->stats.n_class);
      dr.n0 = cur.n0;
      h->arena.release(W);
      h->arena.release(Wi);
      h->arena.release(mrow);
      h->arena.release(desc);

      // ledger (real flops, complex multiply-add = 8) and skeleton export
      std::vector<int> kk(nbox, -1);
      std::vector<int64_t> sid;
      for (int b = 0; b < nbox; ++b) {
        const int n = cur.n0[b];
        if (n == 0) continue;
        const int k = curk[b];
        kk[b] = k;
        for (int i = 0; i < k; ++i) sid.push_back(ids[cur.ioff[b] + i]);
        const double m = dr.m[b], k_ = dr.k[b], r_ = dr.r[b], nN = dr.nN[b];
        flops_id += 4.0 * (4.0 * m * n * k_ - 2.0 * (m + n) * k_ * k_ + 4.0 * k_ * k_ * k_ / 3.0);
        kevals += 2.0 * npx * n;
        if (r_ > 0) {
          flops_lu += 8.0 / 3.0 * r_ * r_ * r_;
          flops_y += 8.0 * r_ * r_ * (k_ + nN);
          flops_schur += 8.0 * (k_ + nN) * (k_ + nN) * r_;
          fbytes += E * (k_ * r_ + r_ * r_ + 2.0 * (k_ + nN) * r_);
          h->stats.boxes_compressed++;
        }
        if (d < 16) {
          h->stats.rank_sum[d] += dr.k[b];
          h->stats.redundant_sum[d] += dr.r[b];
          h->stats.box_count[d] += 1;
        }
      }
      h->skel_k.push_back(kk);
      h->skel_ids.push_back(sid);
      h->recs.push_back(std::move(dr));

      // parent lists: sorted union of the children's skeletons (Fig. f:merge)
      const bool last = (d == MIN_DEPTH);
      if (last) {
        for (int b = 0; b < nbox; ++b)
          for (int i = 0; i < curk[b]; ++i) root_list.push_back({b, i, ids[cur.ioff[b] + i]});
        std::sort(root_list.begin(), root_list.end(),
                  [](const ListEntry& a, const ListEntry& b) { return a.gid < b.gid; });
        break;
      }
      const int pd = d - 1, pnb = 1 << pd, pbox = pnb * pnb;
      std::vector<std::vector<ListEntry>> plist(pbox);
      std::vector<int> pcount(pbox, 0);
      for (int p = 0; p < pbox; ++p) {
        const int px = p % pnb, py = p / pnb;
        for (int j = 0; j < 2; ++j)
          for (int i = 0; i < 2; ++i) {
            const int c = (2 * py + j) * nb + (2 * px + i);
            for (int q = 0; q < curk[c]; ++q) plist[p].push_back({c, q, ids[cur.ioff[c] + q]});
          }
        std::sort(plist[p].begin(), plist[p].end(),
                  [](const ListEntry& a, const ListEntry& b) { return a.gid < b.gid; });
        pcount[p] = (int)plist[p].size();
      }
      LevelHost par;
      par.layout(pd, pcount);
      par.idx.resize(par.ioff.empty() ? 0 : (size_t)(par.ioff.back() + pcount.back()));
      std::vector<ListEntry> lists;
      std::vector<int64_t> loff(pbox);
      for (int p = 0; p < pbox; ++p) {
        loff[p] = (int64_t)lists.size();
        for (size_t q = 0; q < plist[p].size(); ++q) {
          par.idx[par.ioff[p] + q] = plist[p][q].gid;
          lists.push_back(plist[p][q]);
        }
      }
      std::vector<PairDesc> pds;
      for (int p = 0; p < pbox; ++p)
        for (int sl = 0; sl < 25; ++sl) {
          const int64_t off = par.boff[(size_t)p * 25 + sl];
          if (off < 0) continue;
          const int p2 = (p / pnb + sl / 5 - 2) * pnb + (p % pnb + sl % 5 - 2);
          if (pcount[p] == 0 || pcount[p2] == 0) continue;
          PairDesc q;
          q.off = off;
          q.ld = pcount[p];
          q.nr = pcount[p];
          q.nc = pcount[p2];
          q.roff = loff[p];
          q.coff = loff[p2];
          pds.push_back(q);
          // fresh evaluations: child pairs further than distance 2
          const int px = p % pnb, py = p / pnb, qx = p2 % pnb, qy = p2 / pnb;
          for (int a = 0; a < 4; ++a)
            for (int bq = 0; bq < 4; ++bq) {
              const int ca = (2 * py + a / 2) * nb + 2 * px + a % 2;
              const int cb = (2 * qy + bq / 2) * nb + 2 * qx + bq % 2;
              if (chebyshev(nb, ca, cb) > 2) kevals += (double)curk[ca] * curk[cb];
            }
        }
      alloc_level(h, par, E);
      Level<R> child = dev_level<R>(cur, h->x0, h->y0, h->s0);
      PairDesc* d_pds = h->arena.up(pds, s);
      ListEntry* d_lists = h->arena.up(lists, s);
      h->prof.run(RSS_K_ASSEMBLE, s, [&] {
        launch_assemble_pairs<R>(d_pds, (int)pds.size(), d_lists, par.nmax, par.nmax, &child,
                                 (cx<R>*)par.d_A, kp, h->d_P, s);
      });
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      h->arena.release(d_pds);
      h->arena.release(d_lists);
      free_level(h, cur);
      cur = std::move(par);
    }
  } else {
    for (int64_t i = 0; i < N; ++i) root_list.push_back({0, 0, (int)i});
  }

  // root: everything that remains, dense (the top of Alg. a:fact)
  const int nr = (int)root_list.size();
  h->n_root = nr;
  h->stats.n_root = nr;
  if (nr > 0) {
    std::vector<int> rid(nr);
    for (int i = 0; i < nr; ++i) rid[i] = root_list[i].gid;
    h->d_root_ids = h->arena.up(rid, s);
    const size_t bytes = (size_t)nr * nr * E;
    void* A = h->arena.alloc(bytes);
    void* tmp = h->arena.alloc(bytes);
    PairDesc q;
    q.off = 0;
    q.ld = nr;
    q.nr = nr;
    q.nc = nr;
    q.roff = 0;
    q.coff = 0;
    std::vector<PairDesc> pds{q};
    PairDesc* d_pds = h->arena.up(pds, s);
    ListEntry* d_list = h->arena.up(root_list, s);
    Level<R> child{};
    const bool have = D >= MIN_DEPTH;
    if (have) child = dev_level<R>(cur, h->x0, h->y0, h->s0);
    h->prof.run(RSS_K_ASSEMBLE, s, [&] {
      launch_assemble_pairs<R>(d_pds, 1, d_list, nr, nr, have ? &child : nullptr, (cx<R>*)A, kp,
                               h->d_P, s);
    });
    unsigned long long* keys = (unsigned long long*)h->arena.alloc((size_t)nr * 8);
    int* perm = (int*)h->arena.alloc((size_t)nr * 2 * sizeof(int));
    int where = 0;
    h->prof.run(RSS_K_ROOT, s, [&] {
      where = launch_root_inverse<R>((cx<R>*)A, (cx<R>*)tmp, nr, keys, perm, h->d_err, s);
    });
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    h->arena.release(d_pds);
    h->arena.release(d_list);
    h->arena.release(keys);
    h->arena.release(perm);
    if (where == 0) {
      h->d_root_inv = A;
      h->arena.release(tmp);
    } else {
      h->d_root_inv = tmp;
      h->arena.release(A);
    }
    flops_lu += 8.0 * (double)nr * nr * nr;
    fbytes += (double)nr * nr * E;
    if (!have) kevals += (double)nr * nr;
  }
  if (D >= MIN_DEPTH) free_level(h, cur);
  HIPCHK(hipEventRecord(ev1, s));
  HIPCHK(hipEventSynchronize(ev1));
  h->prof.collect(h->stats.t_class_ms, h->stats.n_class);
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  int err = 0;
  HIPCHK(hipMemcpy(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err & ERRF_SINGULAR) fail(RSS_ESINGULAR, "zero pivot in a redundant-block or root inverse");
  h->stats.t_factor_ms = ms;
  h->stats.flops_id = flops_id;
  h->stats.flops_lu = flops_lu;
  h->stats.flops_y = flops_y;
  h->stats.flops_schur = flops_schur;
  h->stats.factor_bytes = fbytes;
  h->stats.kernel_evals = kevals;
  h->d_gemm_desc = h->arena.alloc(sizeof(GemmDesc<R>));
}

// z <- F^{-1} z for z (N x nrhs, complex<R>, ld N) on the handle's stream
template <class R>
void apply_impl(rss_ctx* h, cx<R>* z, int nrhs) {
  hipStream_t s = h->stream;
  const int64_t ldz = h->N;
  const int npx = h->opt.n_proxy;
  const double crad = h->opt.proxy_radius;
  for (auto& dr : h->recs) {
    Records<R> rec = dev_records<R>(dr);
    for (int c = 0; c < 9; ++c) {
      Phase<R> ph = dev_phase<R>(dr.ph[c], nullptr, nullptr, nullptr, npx, crad);
      launch_solve_fwd<R>(ph, rec, z, ldz, nrhs, dr.kmax, dr.rmax, s);
    }
  }
  const int nr = h->n_root;
  if (nr > 0) {
    const size_t need = (size_t)nr * nrhs * sizeof(cx<R>) * 2;
    if (need > h->ws_root_bytes) {
      h->arena.release(h->ws_root);
      h->ws_root = h->arena.alloc(need);
      h->ws_root_bytes = need;
    }
    cx<R>* a = (cx<R>*)h->ws_root;
    cx<R>* b = a + (size_t)nr * nrhs;
    launch_gather_rows<R>(z, ldz, h->d_root_ids, nr, nrhs, a, s);
    GemmDesc<R> d;
    d.C = b;
    d.A = (const cx<R>*)h->d_root_inv;
    d.B = a;
    d.ldc = nr;
    d.lda = nr;
    d.ldb = nr;
    d.M = nr;
    d.N = nrhs;
    d.K = nr;
    d.beta = 0;
    d.sign = 1;
    HIPCHK(hipMemcpyAsync(h->d_gemm_desc, &d, sizeof(d), hipMemcpyHostToDevice, s));
    launch_gemm<R>((GemmDesc<R>*)h->d_gemm_desc, 1, nr, nrhs, s);
    launch_scatter_rows<R>(b, h->d_root_ids, nr, nrhs, z, ldz, s);
    HIPCHK(hipStreamSynchronize(s));  // the descriptor lives on this stack frame
  }
  for (auto it = h->recs.rbegin(); it != h->recs.rend(); ++it) {
    Records<R> rec = dev_records<R>(*it);
    for (int c = 8; c >= 0; --c) {
      Phase<R> ph = dev_phase<R>(it->ph[c], nullptr, nullptr, nullptr, npx, crad);
      launch_solve_bwd<R>(ph, rec, z, ldz, nrhs, it->kmax, it->rmax, it->snmax, s);
    }
  }
  HIPCHK(hipGetLastError());
}

int run(const std::function<void()>& f) {
  try {
    g_err.clear();
    f();
    return RSS_OK;
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return RSS_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return RSS_EHIP;
  }
}

}  // namespace

extern "C" {

int rss_factor_ex(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
                  const rss_options* opt, rss_handle* out) {
  if (out) *out = nullptr;
  rss_ctx* h = nullptr;
  const int rc = run([&] {
    if (!out) fail(RSS_EINVAL, "null output handle pointer");
    validate(points, n, k, tol, leaf);
    h = new rss_ctx();
    h->N = n;
    h->kern = *k;
    h->kp = to_kp(*k);
    h->tol = tol;
    h->leaf = leaf;
    if (opt) h->opt = *opt;
    if (h->opt.n_proxy < 0) fail(RSS_EINVAL, "n_proxy must be >= 0");
    if (h->opt.n_proxy == 0) h->opt.n_proxy = (k->kind == RSS_HELMHOLTZ2D) ? 128 : 64;
    if (!(h->opt.proxy_radius >= 0) || !std::isfinite(h->opt.proxy_radius))
      fail(RSS_EINVAL, "bad proxy_radius");
    if (h->opt.proxy_radius == 0) h->opt.proxy_radius = 1.25;
    if (h->opt.refine_tol == 0) h->opt.refine_tol = 1e-10;
    // refinement steps after the first solve (-1: no refinement, plain apply)
    if (h->opt.precision == RSS_FP32_REFINE)
      h->refine_steps = h->opt.max_refine == 0 ? 10 : (h->opt.max_refine < 0 ? -1 : h->opt.max_refine);
    else
      h->refine_steps = h->opt.max_refine > 0 ? h->opt.max_refine : -1;
    if (h->opt.precision != RSS_FP64 && h->opt.precision != RSS_FP32_REFINE)
      fail(RSS_EINVAL, "unknown precision");
    h->precision = h->opt.precision;
    h->prof.on = h->opt.profile != 0;
    h->stats.precision = h->precision;
    h->stats.n = n;
    h->stats.last_relres = -1.0;
    if (h->opt.stream) {
      h->stream = (hipStream_t)h->opt.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
      h->own_stream = true;
    }
    // root square
    if (h->opt.root[2] > 0) {
      h->x0 = h->opt.root[0];
      h->y0 = h->opt.root[1];
      h->s0 = h->opt.root[2];
    } else {
      double lox = points[0], hix = points[0], loy = points[1], hiy = points[1];
      for (int64_t i = 0; i < n; ++i) {
        lox = std::min(lox, points[2 * i]);
        hix = std::max(hix, points[2 * i]);
        loy = std::min(loy, points[2 * i + 1]);
        hiy = std::max(hiy, points[2 * i + 1]);
      }
      if (lox >= 0 && loy >= 0 && hix <= 1 && hiy <= 1) {
        h->x0 = 0;
        h->y0 = 0;
        h->s0 = 1;
      } else {
        double side = std::max(hix - lox, hiy - loy) * (1.0 + 1e-12);
        if (side == 0) side = 1.0;
        h->x0 = lox;
        h->y0 = loy;
        h->s0 = side;
      }
    }
    h->d_P = (double*)h->arena.alloc((size_t)n * 2 * sizeof(double));
    HIPCHK(hipMemcpyAsync(h->d_P, points, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice,
                          h->stream));
    h->d_err = (int*)h->arena.alloc(sizeof(int));
    HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->stream));
    if (h->precision == RSS_FP64) factor_impl<double>(h, points);
    else factor_impl<float>(h, points);
    h->stats.device_bytes = h->arena.bytes;
  });
  if (rc != RSS_OK) {
    if (h) {
      if (h->own_stream && h->stream) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipStreamDestroy(h->stream);
      }
      delete h;
    }
    return rc;
  }
  *out = h;
  return RSS_OK;
}

int rss_factor(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
               rss_handle* out) {
  return rss_factor_ex(points, n, k, tol, leaf, nullptr, out);
}

int rss_apply(rss_handle h, void* B, int nrhs) {
  return run([&] {
    if (!h || !B) fail(RSS_EINVAL, "null argument");
    if (nrhs < 1) fail(RSS_EINVAL, "nrhs must be >= 1");
    if (h->precision == RSS_FP64) {
      apply_impl<double>(h, (cx<double>*)B, nrhs);
    } else {
      const size_t tot = (size_t)h->N * nrhs;
      cx<float>* z = (cx<float>*)h->arena.alloc(tot * sizeof(cx<float>));
      launch_cast_c64((const cx<double>*)B, h->N, nrhs, z, h->stream);
      // B := 0 + 1 * z
      HIPCHK(hipMemsetAsync(B, 0, tot * sizeof(cx<double>), h->stream));
      apply_impl<float>(h, z, nrhs);
      launch_axpy_from_c64(z, h->N, nrhs, nullptr, (cx<double>*)B, h->stream);
      HIPCHK(hipStreamSynchronize(h->stream));
      h->arena.release(z);
    }
    HIPCHK(hipStreamSynchronize(h->stream));
  });
}

int rss_solve(rss_handle h, void* B, int nrhs) {
  int code = RSS_OK;
  const int rc = run([&] {
    if (!h || !B) fail(RSS_EINVAL, "null argument");
    if (nrhs < 1) fail(RSS_EINVAL, "nrhs must be >= 1");
    hipStream_t s = h->stream;
    const int64_t N = h->N;
    const size_t tot = (size_t)N * nrhs;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    const bool refine = h->refine_steps >= 0;
    h->stats.last_iters = 0;
    if (!refine) {
      if (h->precision == RSS_FP64) {
        apply_impl<double>(h, (cx<double>*)B, nrhs);
      } else {
        cx<float>* z = (cx<float>*)h->arena.alloc(tot * sizeof(cx<float>));
        launch_cast_c64((const cx<double>*)B, N, nrhs, z, s);
        HIPCHK(hipMemsetAsync(B, 0, tot * sizeof(cx<double>), s));
        apply_impl<float>(h, z, nrhs);
        launch_axpy_from_c64(z, N, nrhs, nullptr, (cx<double>*)B, s);
        HIPCHK(hipStreamSynchronize(s));
        h->arena.release(z);
      }
      h->stats.last_relres = -1.0;
    } else {
      cx<double>* b = (cx<double>*)h->arena.alloc(tot * sizeof(cx<double>));
      cx<double>* x = (cx<double>*)h->arena.alloc(tot * sizeof(cx<double>));
      cx<double>* r = (cx<double>*)h->arena.alloc(tot * sizeof(cx<double>));
      double* nrm = (double*)h->arena.alloc((size_t)nrhs * 2 * sizeof(double));
      cx<float>* z = h->precision == RSS_FP32_REFINE
                         ? (cx<float>*)h->arena.alloc(tot * sizeof(cx<float>))
                         : nullptr;
      HIPCHK(hipMemcpyAsync(b, B, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemsetAsync(x, 0, tot * sizeof(cx<double>), s));
      HIPCHK(hipMemcpyAsync(r, B, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
      std::vector<double> bn(nrhs), rn(nrhs);
      launch_colnorms(b, N, nrhs, nrm + nrhs, s);
      HIPCHK(hipMemcpyAsync(bn.data(), nrm + nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double relres = 1.0;
      int it = 0;
      for (;; ++it) {
        // correction d = F^{-1} r, x += d
        if (h->precision == RSS_FP32_REFINE) {
          launch_colnorms(r, N, nrhs, nrm, s);
          launch_scale_to_c64(r, N, nrhs, nrm, z, s);
          apply_impl<float>(h, z, nrhs);
          launch_axpy_from_c64(z, N, nrhs, nrm, x, s);
        } else {
          apply_impl<double>(h, r, nrhs);
          launch_add_c128(x, r, (int64_t)tot, s);
        }
        // r = b - A x (FP64, on the fly)
        launch_residual(h->kp, h->d_P, N, x, b, r, nrhs, s);
        launch_colnorms(r, N, nrhs, nrm, s);
        HIPCHK(hipMemcpyAsync(rn.data(), nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        relres = 0.0;
        for (int j = 0; j < nrhs; ++j) relres = std::max(relres, bn[j] > 0 ? rn[j] / bn[j] : 0.0);
        if (relres <= h->opt.refine_tol || it >= h->refine_steps) break;
      }
      h->stats.last_relres = relres;
      h->stats.last_iters = it;
      HIPCHK(hipMemcpyAsync(B, x, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      h->arena.release(b);
      h->arena.release(x);
      h->arena.release(r);
      h->arena.release(nrm);
      if (z) h->arena.release(z);
      if (relres > h->opt.refine_tol) {
        g_err = "refinement did not reach refine_tol";
        code = RSS_ENOCONV;
      }
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    h->stats.t_solve_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
  return rc != RSS_OK ? rc : code;
}

void rss_free(rss_handle h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  const bool own = h->own_stream;
  hipStream_t s = h->stream;
  delete h;
  if (own && s) (void)hipStreamDestroy(s);
}

int rss_info(rss_handle h, rss_stats* s) {
  if (!h || !s) {
    g_err = "null argument";
    return RSS_EINVAL;
  }
  *s = h->stats;
  s->device_bytes = h->arena.bytes;
  return RSS_OK;
}

int rss_skeletons(rss_handle h, int depth, int32_t* counts, int64_t* ids, int64_t cap,
                  int64_t* total) {
  return run([&] {
    if (!h || !counts || !total) fail(RSS_EINVAL, "null argument");
    const int i = h->D - depth;
    if (depth < MIN_DEPTH || i < 0 || i >= (int)h->skel_k.size()) fail(RSS_EINVAL, "depth not compressed");
    const auto& kk = h->skel_k[i];
    const auto& sid = h->skel_ids[i];
    for (size_t b = 0; b < kk.size(); ++b) counts[b] = kk[b];
    *total = (int64_t)sid.size();
    if (ids) {
      if (cap < (int64_t)sid.size()) fail(RSS_EINVAL, "ids capacity too small");
      std::memcpy(ids, sid.data(), sid.size() * sizeof(int64_t));
    }
  });
}

int rss_kernel_block(const rss_kernel* k, const double* points, int64_t n, const int32_t* I,
                     int64_t ni, const int32_t* J, int64_t nj, void* out, void* stream) {
  return run([&] {
    if (!k || !points || !I || !J || !out) fail(RSS_EINVAL, "null argument");
    if (n < 1 || ni < 0 || nj < 0) fail(RSS_EINVAL, "bad sizes");
    const KParams kp = to_kp(*k);
    launch_kernel_block(kp, points, I, ni, J, nj, (cx<double>*)out, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  });
}

int rss_residual(const rss_kernel* k, const double* points, int64_t n, const void* X, const void* B,
                 void* R, int nrhs, void* stream) {
  return run([&] {
    if (!k || !points || !X || !B || !R) fail(RSS_EINVAL, "null argument");
    if (n < 1 || nrhs < 1) fail(RSS_EINVAL, "bad sizes");
    const KParams kp = to_kp(*k);
    launch_residual(kp, points, n, (const cx<double>*)X, (const cx<double>*)B, (cx<double>*)R, nrhs,
                    (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  });
}

const char* rss_last_error(void) { return g_err.c_str(); }

const char* rss_error_string(int code) {
  switch (code) {
    case RSS_OK: return "RSS_OK";
    case RSS_EINVAL: return "RSS_EINVAL";
    case RSS_ENOMEM: return "RSS_ENOMEM";
    case RSS_EUNSUPPORTED: return "RSS_EUNSUPPORTED";
    case RSS_ESINGULAR: return "RSS_ESINGULAR";
    case RSS_ENOCONV: return "RSS_ENOCONV";
    case RSS_EHIP: return "RSS_EHIP";
    default: return "RSS_UNKNOWN";
  }
}

}  // extern "C"
