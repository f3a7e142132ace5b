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
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <exception>
#include <limits>
#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "rss.h"
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

// Requests up to SMALL bytes are carved from SLAB-byte blocks, one hipMalloc
// per block; larger ones get their own allocation.  Carved pieces live as long
// as their owner (release() ignores them).
constexpr size_t SLAB = (size_t)2 << 20, SMALL = (size_t)64 << 10;

// Device memory cache.  Freed blocks stay with the library, per device and
// size class (four classes per power of two), and are handed out again, so
// the per-depth stores of a factorization and repeated factorizations do not
// pay a hipMalloc and a device-synchronizing hipFree per block.  Callers free
// only memory that no queued work uses any more (every free follows a
// synchronization of the stream that used it; when an error unwinds an
// operation, the device is synchronized before its blocks are cached).  Up to
// three quarters of the device's memory is kept cached (a batched
// factorization of a few hundred problems reuses its ~100 GB of blocks instead
// of mapping them again on every call); a block freed past that goes back to
// the driver.  hipFree synchronizes the device, so a cache filled with another
// workload's blocks slows the next large factorization (its frees past the
// cap stall the host's pipelined launches): a caller switching to a different
// workload calls rss_trim_cache first.  When an allocation fails, the largest
// cached blocks go back until the request's size (and half again) is
// released, then the whole cache if that was not enough.
class DevPool {
 public:
  void* alloc(size_t n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t c = size_class(n);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto& fl = free_[{dev, c}];
      if (!fl.empty()) {
        void* p = fl.back();
        fl.pop_back();
        cached_[dev] -= c;
        live_[p] = {dev, c};
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
      // give back the largest cached blocks, about what the request needs
      // (unmapping the whole cache can take seconds), then all of them
      (void)hipGetLastError();
      trim(dev, c + c / 2);
      if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        trim(dev);
        if (hipMalloc(&p, c) != hipSuccess) {
          (void)hipGetLastError();
          return nullptr;
        }
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = {dev, c};
    return p;
  }
  void free(void* p) {
    if (!p) return;
    if (std::uncaught_exceptions() > 0) (void)hipDeviceSynchronize();
    std::unique_lock<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) {
      g.unlock();
      (void)hipFree(p);
      return;
    }
    const int dev = it->second.first;
    const size_t c = it->second.second;
    live_.erase(it);
    if (cached_[dev] + c <= cap(dev)) {
      free_[{dev, c}].push_back(p);
      cached_[dev] += c;
      return;
    }
    g.unlock();
    (void)hipFree(p);
  }

 private:
  static size_t size_class(size_t n) {
    size_t b = 1;
    while (b * 2 <= n) b *= 2;
    const size_t step = b >= 4 ? b / 4 : 1;
    return (n + step - 1) / step * step;
  }
  size_t cap(int dev) {  // with mu_ held
    auto it = cap_.find(dev);
    if (it != cap_.end()) return it->second;
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    return cap_[dev] = tot / 4 * 3;
  }

 public:
  // return device dev's cached blocks to the driver, largest first, until at
  // least `want` bytes are released (all of them by default); the bytes
  // released
  size_t trim(int dev, size_t want = ~(size_t)0) {
    std::vector<void*> out;
    size_t bytes = 0;
    {
      std::lock_guard<std::mutex> g(mu_);
      for (auto it = free_.rbegin(); it != free_.rend() && bytes < want; ++it) {
        if (it->first.first != dev) continue;
        auto& fl = it->second;
        while (!fl.empty() && bytes < want) {
          out.push_back(fl.back());
          fl.pop_back();
          bytes += it->first.second;
        }
      }
      cached_[dev] -= bytes;
    }
    for (void* q : out) (void)hipFree(q);
    return bytes;
  }

 private:
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_;
  std::unordered_map<void*, std::pair<int, size_t>> live_;
  std::map<int, size_t> cached_, cap_;
};

DevPool& pool() {
  static DevPool* p = new DevPool();  // never destroyed: handles may outlive static destruction order
  return *p;
}

void* dev_alloc(size_t n) {
  void* p = pool().alloc(n);
  if (!p) fail(RSS_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
  return p;
}

void dev_free(void* p) { pool().free(p); }

struct Carver {
  std::vector<void*> slabs;
  size_t used = SLAB;
  void* take(size_t n, double& bytes) {
    n = (n + 255) & ~(size_t)255;
    if (used + n > SLAB) {
      slabs.push_back(dev_alloc(SLAB));
      bytes += (double)SLAB;
      used = 0;
    }
    void* p = (char*)slabs.back() + used;
    used += n;
    return p;
  }
  void clear() {
    for (void* p : slabs) dev_free(p);
    slabs.clear();
    used = SLAB;
  }
};

// device memory owned by a handle
struct Arena {
  std::vector<void*> ptrs;    // own allocations (large requests)
  std::vector<size_t> sizes;  // parallel to ptrs
  Carver small;
  double bytes = 0;
  void* alloc(size_t n) {
    if (n == 0) n = 16;
    if (n <= SMALL) return small.take(n, bytes);
    void* p = dev_alloc(n);
    ptrs.push_back(p);
    sizes.push_back(n);
    bytes += (double)n;
    return p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      dev_free(p);
      const size_t i = (size_t)(it - ptrs.begin());
      bytes -= (double)sizes[i];
      ptrs.erase(it);
      sizes.erase(sizes.begin() + (long)i);
    }
  }
  ~Arena() {
    for (void* p : ptrs) dev_free(p);
    small.clear();
  }
  template <class T>
  T* up(const std::vector<T>& v, hipStream_t s) {
    T* p = (T*)alloc(v.size() * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
};

// Gathers small host arrays into one staging buffer (256-byte aligned pieces)
// that flush() uploads with a single copy into one device block from the given
// allocator, then points every registered destination into that block.
// Destinations must stay where they are until flush().
struct Packer {
  std::vector<char> buf;
  std::vector<std::pair<void**, size_t>> refs;
  size_t reserve(size_t bytes) {
    const size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + std::max<size_t>(bytes, 16), 0);
    return off;
  }
  template <class T, class U>
  void add(T*& dst, const std::vector<U>& v) {
    static_assert(std::is_same<typename std::remove_const<T>::type, U>::value, "element type");
    const size_t off = reserve(v.size() * sizeof(U));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(U));
    refs.emplace_back((void**)&dst, off);
  }
  template <class T>
  void zeros(T*& dst, size_t n) {
    refs.emplace_back((void**)&dst, reserve(n * sizeof(T)));
  }
  template <class A>
  void* flush(A& alloc, hipStream_t s) {
    if (refs.empty()) return nullptr;
    char* d = (char*)alloc.alloc(buf.size());
    HIPCHK(hipMemcpyAsync(d, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
    for (auto& r : refs) *r.first = d + r.second;
    buf.clear();
    refs.clear();
    return d;
  }
};

// page-locked host buffer for readbacks; grows on demand
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
  void* get(size_t n) {
    if (n > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      n = std::max(n, (size_t)1 << 20);
      HIPCHK(hipHostMalloc(&p, n, hipHostMallocDefault));
      cap = n;
    }
    return p;
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
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
  void* d_blk = nullptr;  // one block holding d_n0 .. d_boff
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
  std::vector<int> boxes;  // boxes of one colour, ascending id
  int* d_box = nullptr;
  int* d_prob = nullptr;   // all zero: the single-problem solve
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
  int kmax = 0, rmax = 0, qmax = 0, snmax = 0;
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

// a captured apply of one handle (see ApplyGraph); destroyed with the handle
struct ApplyGraphBase {
  uint64_t last_use = 0;  // for the handle's least-recently-used eviction
  virtual ~ApplyGraphBase() {}
};

// Product with A on a uniform grid by FFT (launch_grid_apply): the generator's
// transform, the point scales and diagonal, and a work array grown on demand.
struct rss_gridop {
  GridDesc g{};
  rss_kernel kern{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cx<double>* ghat = nullptr;
  cx<double>* tw = nullptr;
  double* scale = nullptr;
  cx<double>* diag = nullptr;
  cx<double>* work = nullptr;
  size_t work_elems = 0;
  ~rss_gridop() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : {(void*)ghat, (void*)tw, (void*)scale, (void*)diag, (void*)work})
      if (p) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  // Y = A X (mode 0) or B - A X (mode 1) on stream st; ld = n^2; columns in
  // chunks of at most 16 (the work array holds one chunk)
  void apply(const cx<double>* X, const cx<double>* B, cx<double>* Y, int nrhs, int mode, hipStream_t st) {
    constexpr int CH = 16;
    const int64_t ld = (int64_t)g.n * g.n;
    const size_t need = (size_t)std::min(nrhs, CH) * g.n * g.M;
    if (need > work_elems) {
      HIPCHK(hipStreamSynchronize(st));
      if (work) HIPCHK(hipFree(work));
      work = nullptr;
      work_elems = 0;
      HIPCHK(hipMalloc((void**)&work, need * sizeof(cx<double>)));
      work_elems = need;
    }
    for (int c0 = 0; c0 < nrhs; c0 += CH)
      launch_grid_apply(g, X + c0 * ld, B ? B + c0 * ld : nullptr, Y + c0 * ld, ld, std::min(CH, nrhs - c0),
                        work, mode, st);
  }
  double device_bytes() const {
    return (double)g.M * g.M * 16 + (double)g.M * 8 + (double)g.n * g.n * 24 + (double)work_elems * 16;
  }
};

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
  std::shared_ptr<void> stream_owner;  // destroys a library-created stream with its last handle
  double x0 = 0, y0 = 0, s0 = 1;
  int D = 0;
  Arena arena;
  double* d_P = nullptr;
  int* d_tperm = nullptr;  // residual target order (spatial_order), made on the first refined solve
  std::vector<DepthRecords> recs;  // index 0 .. : depths D, D-1, ..., 2
  int n_root = 0;
  int* d_root_ids = nullptr;
  void* d_root_inv = nullptr;
  void* root_spare = nullptr;
  std::vector<double> h_points;     // host copy of the points (planner)
  std::vector<LevelHost> tmp_levels;
  std::vector<int64_t> skel_counts_off;
  std::vector<std::vector<int>> skel_k;          // per compressed depth: k per box (-1 empty)
  std::vector<std::vector<int64_t>> skel_ids;    // per compressed depth: concatenated ids
  rss_stats stats{};
  Prof prof;
  int* d_err = nullptr;
  rss_gridop* gridop = nullptr;  // refinement residual by FFT (rss_set_residual_op), not owned
  bool no_mg = false;            // factor without the multi-workgroup QR (after a barrier timeout)
  // captured applies per (sizeof(R), nrhs), at most MAX_GRAPHS (least recently
  // used dropped); declared last, so destroyed before the arena that owns the
  // factors they read
  static constexpr size_t MAX_GRAPHS = 4;
  std::map<std::pair<int, int>, std::unique_ptr<ApplyGraphBase>> graphs;
  uint64_t graph_clock = 0;
};

namespace {

// Integral of K over the h x h cell centred at the origin (eqs. e:a1i, e:b2).
// The square is 8 congruent triangles 0 <= t <= pi/4, 0 <= r <= a / cos t
// (a = h/2), so c = 8 int_0^{pi/4} F(a / cos t) dt with F(rho) = int_0^rho K(r) r dr:
//  Laplace K = -log(r)/(2 pi): F(rho) = -(rho^2 log rho / 2 - rho^2 / 4) / (2 pi)
//    and, in closed form, c = -(a^2/pi) (2 log a + log 2 - 3 + pi/2);
//  Helmholtz K = (i/4) H0^(1)(kappa r): d/dz [z H1(z)] = z H0(z) and z H1(z) -> -2i/pi,
//    so F(rho) = (i/4) (rho H1(kappa rho) / kappa + 2i / (pi kappa^2)); the smooth
//    integral over t by 64-point Gauss-Legendre quadrature.
std::complex<double> cell_integral(const rss_kernel& k) {
  const double a = 0.5 * k.h;
  if (k.kind == RSS_LAPLACE2D)
    return {-(a * a / M_PI) * (2.0 * std::log(a) + std::log(2.0) - 3.0 + 0.5 * M_PI), 0.0};
  constexpr int NG = 64;
  double sum_re = 0.0, sum_im = 0.0;
  for (int i = 1; i <= NG; ++i) {
    // i-th root of the Legendre polynomial P_NG by Newton's method
    double x = std::cos(M_PI * (i - 0.25) / (NG + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= NG; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = NG * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    const double wgt = 2.0 / ((1.0 - x * x) * dp * dp);
    const double t = 0.125 * M_PI * (x + 1.0);  // [-1, 1] -> [0, pi/4]
    const double rho = a / std::cos(t), z = k.kappa * rho;
    const double j1 = std::cyl_bessel_j(1.0, z), y1 = std::cyl_neumann(1.0, z);
    // (i/4) (rho (j1 + i y1) / kappa + 2i / (pi kappa^2))
    const double in_re = rho * j1 / k.kappa, in_im = rho * y1 / k.kappa + 2.0 / (M_PI * k.kappa * k.kappa);
    sum_re += wgt * (-0.25 * in_im);
    sum_im += wgt * (0.25 * in_re);
  }
  const double scale = 8.0 * 0.125 * M_PI;  // 8 triangles, dt = (pi/8) dx
  return {scale * sum_re, scale * sum_im};
}

KParams to_kp(const rss_kernel& k) {
  KParams p;
  p.kind = (int)k.kind;
  p.q = k.q;
  p.kappa = k.kappa;
  p.weight = k.weight;
  p.diag = k.diag;
  p.bump = k.bump_a > 0 ? 1 : 0;
  p.bump_a = k.bump_a;
  p.bcx = k.bump_c[0];
  p.bcy = k.bump_c[1];
  p.cdre = p.cdim = 0.0;
  if (k.cell_diag) {
    const std::complex<double> c = cell_integral(k) * (k.weight / (k.h * k.h));
    p.cdre = c.real();
    p.cdim = c.imag();
  }
  return p;
}

// Equal points share a cell of a 2^15 x 2^15 grid over their bounding box.
// The (cell key, index) pairs are sorted by key -- a linear scan when they
// already are (points listed cell by cell, e.g. a grid in row order), else
// three 10-bit radix passes -- and the points of each cell compared exactly.
void check_distinct(const double* points, int64_t n) {
  if (n < 2) return;
  double x0 = points[0], x1 = points[0], y0 = points[1], y1 = points[1];
  for (int64_t i = 1; i < n; ++i) {
    x0 = std::min(x0, points[2 * i]);
    x1 = std::max(x1, points[2 * i]);
    y0 = std::min(y0, points[2 * i + 1]);
    y1 = std::max(y1, points[2 * i + 1]);
  }
  constexpr int B = 15, NB = 1 << B;
  const double sx = x1 > x0 ? (double)NB / (x1 - x0) : 0.0, sy = y1 > y0 ? (double)NB / (y1 - y0) : 0.0;
  std::vector<uint64_t> a((size_t)n);
  bool sorted = true;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t cx = (uint64_t)std::min<double>(NB - 1, std::floor((points[2 * i] - x0) * sx));
    const uint64_t cy = (uint64_t)std::min<double>(NB - 1, std::floor((points[2 * i + 1] - y0) * sy));
    a[(size_t)i] = (((cy << B) | cx) << 32) | (uint64_t)i;
    if (i > 0 && (a[(size_t)i] >> 32) < (a[(size_t)i - 1] >> 32)) sorted = false;
  }
  if (!sorted) {
    constexpr int RB = 10, NR = 1 << RB;
    std::vector<uint64_t> b((size_t)n);
    std::vector<uint32_t> cnt(NR + 1);
    for (int pass = 0; pass < 3; ++pass) {
      std::fill(cnt.begin(), cnt.end(), 0u);
      const int sh = 32 + pass * RB;
      for (int64_t i = 0; i < n; ++i) cnt[((a[(size_t)i] >> sh) & (NR - 1)) + 1]++;
      for (int d = 0; d < NR; ++d) cnt[d + 1] += cnt[d];
      for (int64_t i = 0; i < n; ++i) b[cnt[(a[(size_t)i] >> sh) & (NR - 1)]++] = a[(size_t)i];
      a.swap(b);
    }
  }
  for (int64_t lo = 0; lo < n;) {
    int64_t hi = lo + 1;
    while (hi < n && (a[(size_t)hi] >> 32) == (a[(size_t)lo] >> 32)) ++hi;
    if (hi - lo > 1) {
      std::vector<int64_t> run;
      for (int64_t i = lo; i < hi; ++i) run.push_back((int64_t)(a[(size_t)i] & 0xffffffffu));
      std::sort(run.begin(), run.end(), [points](int64_t u, int64_t v) {
        if (points[2 * u] != points[2 * v]) return points[2 * u] < points[2 * v];
        if (points[2 * u + 1] != points[2 * v + 1]) return points[2 * u + 1] < points[2 * v + 1];
        return u < v;
      });
      for (size_t i = 1; i < run.size(); ++i) {
        const int64_t u = run[i - 1], v = run[i];
        if (points[2 * u] == points[2 * v] && points[2 * u + 1] == points[2 * v + 1])
          fail(RSS_EINVAL, "duplicate points " + std::to_string(std::min(u, v)) + " and " +
                               std::to_string(std::max(u, v)));
      }
    }
    lo = hi;
  }
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
  if (k->cell_diag && (k->kind == RSS_DEGENERATE || !(k->h > 0) || !std::isfinite(k->h)))
    fail(RSS_EINVAL, "cell_diag needs the Laplace or Helmholtz kernel and h > 0");
  if (!(k->bump_a >= 0) || !std::isfinite(k->bump_a) || !std::isfinite(k->bump_c[0]) ||
      !std::isfinite(k->bump_c[1]))
    fail(RSS_EINVAL, "bad scattering potential parameters");
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(points[i])) fail(RSS_EINVAL, "non-finite point coordinate");
  // coincident points would put K(0) (log 0, H0(0)) into the matrix: reject any repeat
  check_distinct(points, n);
}

// Box coordinates at depth MAX_DEPTH: floor((p - corner) / side) clamped to the
// grid.  The rounded quotient at depth d is 2^d times the one at depth 0
// exactly (a power-of-two scaling), so the box coordinate at depth d is this
// value shifted right by MAX_DEPTH - d.
void grid_coords(const double* P, int64_t n, double x0, double y0, double s0, std::vector<int>& gx,
                 std::vector<int>& gy) {
  const int nb = 1 << MAX_DEPTH;
  const double s = s0 / (double)nb;
  gx.resize(n);
  gy.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    long bx = (long)std::floor((P[2 * i] - x0) / s);
    long by = (long)std::floor((P[2 * i + 1] - y0) / s);
    gx[i] = (int)std::min<long>(std::max<long>(bx, 0), nb - 1);
    gy[i] = (int)std::min<long>(std::max<long>(by, 0), nb - 1);
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

// d_cur and d_idx are adjacent so that one copy reads both back
void alloc_level(rss_ctx* h, LevelHost& L, size_t elem, hipStream_t s) {
  Packer pk;
  pk.add(L.d_n0, L.n0);
  pk.add(L.d_cur, L.n0);
  pk.add(L.d_idx, L.idx);
  pk.add(L.d_ioff, L.ioff);
  pk.add(L.d_boff, L.boff);
  L.d_blk = pk.flush(h->arena, s);
  L.d_A = h->arena.alloc((size_t)L.nA * elem);
}

void free_level(rss_ctx* h, LevelHost& L) {
  h->arena.release(L.d_blk);
  h->arena.release(L.d_A);
  L.d_n0 = L.d_cur = L.d_idx = nullptr;
  L.d_ioff = L.d_boff = nullptr;
  L.d_blk = L.d_A = nullptr;
}

// temporary device buffers of one batched operation; clear() (after the
// stream has drained) frees the large ones and keeps the slabs for reuse
struct Scratch {
  std::vector<void*> ptrs;
  std::vector<void*> slabs;
  size_t si = 0, used = 0;  // current slab and offset in it
  void* alloc(size_t n) {
    if (n == 0) n = 16;
    if (n <= SMALL) {
      n = (n + 255) & ~(size_t)255;
      if (si < slabs.size() && used + n > SLAB) {
        ++si;
        used = 0;
      }
      if (si == slabs.size()) slabs.push_back(dev_alloc(SLAB));
      void* p = (char*)slabs[si] + used;
      used += n;
      return p;
    }
    void* p = dev_alloc(n);
    ptrs.push_back(p);
    return p;
  }
  template <class T>
  T* up(const std::vector<T>& v, hipStream_t s) {
    T* p = (T*)alloc(v.size() * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  void clear() {
    for (void* p : ptrs) dev_free(p);
    ptrs.clear();
    si = 0;
    used = 0;
  }
  void release_all() {
    clear();
    for (void* p : slabs) dev_free(p);
    slabs.clear();
  }
  ~Scratch() { release_all(); }
};

// Largest box (points) whose ID goes through the Gram matrix; larger boxes
// take column-pivoted Householder QR.  GRAM_NMAX unless the environment
// variable RSS_GRAM_NMAX (read once) sets a smaller value (0: Householder QR
// everywhere; for tests that cover both forms).
int gram_nmax() {
  static const int v = [] {
    const char* e = std::getenv("RSS_GRAM_NMAX");
    if (!e || !*e) return GRAM_NMAX;
    return std::max(0, std::min(GRAM_NMAX, std::atoi(e)));
  }();
  return v;
}

std::atomic<bool> g_autotune{true};
std::atomic<int> g_autotune_mode{1};
}  // namespace
namespace rss {
extern thread_local bool g_server_thread;
}
namespace {

// Factor-tile autotuner.  The Gram kernel of the ID splits each box's rows of
// Y = [A_MB; K(proxy, B)] into chunks, one workgroup each (partial Gram
// matrices summed in chunk order); how many pays depends on the number of
// boxes in the launch, their size and their row count.  Per bucket of those
// (precision, box size in steps of 16, log2 of boxes per launch, log2 of rows)
// the first phase that meets it times the candidates (a target of 512 ... 8192
// workgroups per launch) and keeps the fastest for the process; later phases
// of the bucket reuse it.  The kernel is a pure function of the level, so the
// candidates run on the real data and the chosen one runs last.  Off (or in
// the solve server's threads): 2048.
struct GramTuneKey {
  int prec, nb, sb, rb;
  bool operator<(const GramTuneKey& o) const {
    return std::tie(prec, nb, sb, rb) < std::tie(o.prec, o.nb, o.sb, o.rb);
  }
};
struct GramTuneVal {
  int target;   // workgroups per launch aimed at
  int chunks;   // row chunks per box that gave
  float us;     // its time per launch
};
std::mutex g_gram_tune_mu;
std::map<GramTuneKey, GramTuneVal> g_gram_tune;
constexpr int GRAM_TUNE_DEFAULT = 2048;
constexpr int GRAM_TUNE_TARGETS[] = {512, 1024, 2048, 4096, 8192};

int ceil_log2(int v) {
  int b = 0;
  while ((1 << b) < v) ++b;
  return b;
}
GramTuneKey gram_tune_key(int prec_bytes, int nmax, int nslot, int rows_ub) {
  return {prec_bytes, (nmax + 15) / 16, ceil_log2(std::max(1, nslot)), ceil_log2(std::max(1, rows_ub))};
}
// row chunks per box for a target workgroup count: at least 32 rows of Y per
// chunk, chunk rows a multiple of 16
void gram_chunking(int target, int nslot, int nmax, int rows_ub, int& chunks, int& chunk_rows) {
  const int tgroups = gram_tile_groups(std::max(1, nmax));
  const int want = std::max(1, (target + nslot * tgroups - 1) / (nslot * tgroups));
  const int most = std::max(1, (rows_ub + 31) / 32);
  const int ch = std::min(want, most);
  chunk_rows = ((rows_ub + ch - 1) / ch + 15) / 16 * 16;
  chunks = std::max(1, (rows_ub + chunk_rows - 1) / chunk_rows);
}
bool gram_tuning_on() { return g_autotune.load() && g_autotune_mode.load() == 1 && !rss::g_server_thread; }

// Colour of box b (row-major id on an nb x nb grid) in the elimination
// schedule: nine colours (bx mod 3) + 3 (by mod 3), boxes of a colour 3 apart;
// four colours (bx mod 2) + 2 (by mod 2), boxes of a colour 2 apart.
int box_colour(int b, int nb, int colours) {
  const int bx = b % nb, by = b / nb;
  return colours == 4 ? (bx & 1) + 2 * (by & 1) : bx % 3 + 3 * (by % 3);
}
// Four colours: the Schur updates of a colour go in four ordered passes,
// boxes of a pass 4 apart, so no two updates of a pass meet on a block.
int schur_pass(int b, int nb) {
  const int bx = b % nb, by = b / nb;
  return ((bx >> 1) & 1) + 2 * ((by >> 1) & 1);
}

// Bounded wait of the multi-workgroup QR's per-box barriers (spins of about
// 0.1 us); the environment variable RSS_MG_SPIN_LIMIT (read once) sets another
// value (tests force timeouts with a tiny one).
unsigned mg_spin_limit() {
  static const unsigned v = [] {
    const char* e = std::getenv("RSS_MG_SPIN_LIMIT");
    if (!e || !*e) return 1u << 24;
    const long x = std::atol(e);
    return (unsigned)std::max(1L, std::min(x, (long)(1u << 30)));
  }();
  return v;
}

// A per-box barrier of the multi-workgroup QR gave up (other streams kept its
// workgroups from being resident together); the factorization is redone
// without that kernel.
struct MgTimeout {};

// Per-problem state while a batch is being factored.
struct Work {
  rss_ctx* h = nullptr;
  std::vector<int> bo;        // leaf box of every point
  LevelHost cur;
  bool active = false;        // has a level at the current height
  std::vector<ListEntry> root_list;
  double flops_id = 0, flops_lu = 0, flops_y = 0, flops_schur = 0, fbytes = 0, kevals = 0;
};

std::vector<ListEntry> sorted_union(const std::vector<int>& boxes, const std::vector<int>& curk,
                                    const std::vector<int>& ids, const std::vector<int64_t>& ioff) {
  std::vector<ListEntry> out;
  for (int c : boxes)
    for (int q = 0; q < curk[c]; ++q) out.push_back({c, q, ids[ioff[c] + q]});
  std::sort(out.begin(), out.end(), [](const ListEntry& a, const ListEntry& b) { return a.gid < b.gid; });
  return out;
}

// r_p = b_p - A_p x_p for every problem in one batched launch per 16 columns
struct ResProblem {
  KParams kp;
  const double* P;
  int64_t n;
  const cx<double>* X;
  const cx<double>* B;
  cx<double>* R;
  int nrhs;
  const int* tperm;  // device target order, or null (index order)
};

// Points ordered cell by cell (row-major cells of ~64 points over the
// bounding box, index order inside a cell): consecutive runs of 64 targets are
// spatially compact, so the residual's per-pair branch (near / far argument of
// the kernel) takes one side for most waves.
std::vector<int> spatial_order(const double* P, int64_t n) {
  double lox = P[0], hix = P[0], loy = P[1], hiy = P[1];
  for (int64_t i = 1; i < n; ++i) {
    lox = std::min(lox, P[2 * i]);
    hix = std::max(hix, P[2 * i]);
    loy = std::min(loy, P[2 * i + 1]);
    hiy = std::max(hiy, P[2 * i + 1]);
  }
  const int G = std::max(1, (int)std::sqrt((double)n / 64.0));
  const double wx = hix > lox ? (hix - lox) : 1.0, wy = hiy > loy ? (hiy - loy) : 1.0;
  std::vector<int> cell(n), cnt((size_t)G * G + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int cx = std::min(G - 1, std::max(0, (int)((P[2 * i] - lox) / wx * G)));
    const int cy = std::min(G - 1, std::max(0, (int)((P[2 * i + 1] - loy) / wy * G)));
    cell[i] = cy * G + cx;
    cnt[cell[i] + 1]++;
  }
  for (size_t c = 1; c < cnt.size(); ++c) cnt[c] += cnt[c - 1];
  std::vector<int> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[cnt[cell[i]]++] = (int)i;
  return perm;
}

void residual_batch(const std::vector<ResProblem>& rp, Scratch& scr, hipStream_t s) {
  int64_t tblocks = 0;
  int max_nrhs = 0;
  for (const auto& q : rp) {
    tblocks += (q.n + 255) / 256;
    max_nrhs = std::max(max_nrhs, q.nrhs);
  }
  const int S = residual_slices(tblocks);
  std::vector<ResDesc> d(rp.size());
  std::vector<ResBlock> blk, sum_blk;
  for (size_t p = 0; p < rp.size(); ++p) {
    const ResProblem& q = rp[p];
    const int64_t nt = (q.n + 255) / 256;
    ResDesc& e = d[p];
    e.kp = q.kp;
    e.P = q.P;
    e.n = q.n;
    e.X = q.X;
    e.B = q.B;
    e.R = q.R;
    e.nrhs = q.nrhs;
    e.tperm = q.tperm;
    e.S = (int)std::min<int64_t>(S, nt);
    e.part = e.S > 1 ? (cx<double>*)scr.alloc((size_t)e.S * 16 * q.n * sizeof(cx<double>)) : nullptr;
    for (int64_t tb = 0; tb < nt; ++tb) {
      for (int sp = 0; sp < e.S; ++sp) blk.push_back({(int)p, (int)tb, sp});
      if (e.S > 1) sum_blk.push_back({(int)p, (int)tb, 0});
    }
  }
  const ResDesc* dd = scr.up(d, s);
  const ResBlock* db = scr.up(blk, s);
  const ResBlock* ds = sum_blk.empty() ? nullptr : scr.up(sum_blk, s);
  launch_residual(dd, db, (int)blk.size(), ds, (int)sum_blk.size(), max_nrhs, s);
}

// Batched RS-S factorization (Alg. a:fact) of every handle in H, all on stream s.
// Heights above the leaves are aligned: at height t every problem with
// D - t >= 2 eliminates its boxes of depth D - t, colour by colour, and each
// colour is one launch per step over the boxes of all those problems.
template <class R>
void factor_batch(std::vector<rss_ctx*>& H, hipStream_t s) {
  const size_t E = sizeof(cx<R>);
  const int np = (int)H.size();
  std::vector<Work> W(np);
  Prof& prof = H[0]->prof;
  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, s));
  int tmax = -1;
  int* d_err = H[0]->d_err;
  for (int p = 0; p < np; ++p) {
    rss_ctx* h = H[p];
    W[p].h = h;
    // grid coordinates at depth MAX_DEPTH once; a coarser depth is a shift of them
    std::vector<int> gx, gy;
    grid_coords(h->h_points.data(), h->N, h->x0, h->y0, h->s0, gx, gy);
    int D = 0;
    for (;; ++D) {
      if (D > MAX_DEPTH) fail(RSS_EUNSUPPORTED, "tree deeper than 15 levels");
      std::vector<int>& bo = W[p].bo;
      bo.resize(h->N);
      const int sh = MAX_DEPTH - D;
      for (int64_t i = 0; i < h->N; ++i) bo[i] = ((gy[i] >> sh) << D) + (gx[i] >> sh);
      std::vector<int> cnt((size_t)1 << (2 * D), 0);
      int mx = 0;
      for (int64_t i = 0; i < h->N; ++i) mx = std::max(mx, ++cnt[bo[i]]);
      if (mx <= h->leaf) break;
    }
    h->D = D;
    h->stats.depth = D;
    if (D >= MIN_DEPTH) {
      tmax = std::max(tmax, D - MIN_DEPTH);
      const int nbox = 1 << (2 * D);
      std::vector<int> counts(nbox, 0);
      for (int64_t i = 0; i < h->N; ++i) counts[W[p].bo[i]]++;
      LevelHost& L = W[p].cur;
      L.layout(D, counts);
      L.idx.assign(h->N, 0);
      std::vector<int64_t> fillp(L.ioff);
      for (int64_t i = 0; i < h->N; ++i) L.idx[fillp[W[p].bo[i]]++] = (int)i;
      alloc_level(h, L, E, s);
      W[p].active = true;
      W[p].kevals += (double)L.nA;
    } else {
      for (int64_t i = 0; i < h->N; ++i) W[p].root_list.push_back({0, 0, (int)i});
    }
  }
  Scratch scr;
  PinnedBuf pinned;
  // leaf stencils of every problem: one launch
  {
    std::vector<Prob<R>> probs;
    int maxb = 0, lnmax = 0;
    for (int p = 0; p < np; ++p)
      if (W[p].active) {
        Prob<R> pr{};
        pr.L = dev_level<R>(W[p].cur, H[p]->x0, H[p]->y0, H[p]->s0);
        pr.kp = H[p]->kp;
        pr.P = H[p]->d_P;
        probs.push_back(pr);
        maxb = std::max(maxb, W[p].cur.nb * W[p].cur.nb);
        lnmax = std::max(lnmax, W[p].cur.nmax);
      }
    if (!probs.empty()) {
      Prob<R>* d = scr.up(probs, s);
      prof.run(RSS_K_ASSEMBLE, s, [&] { launch_leaf_assemble<R>(d, (int)probs.size(), maxb, lnmax, s); });
    }
  }
  for (int t = 0; t <= tmax; ++t) {
    // problems eliminating at this height, their depth records and device descriptors
    std::vector<int> act;
    for (int p = 0; p < np; ++p)
      if (W[p].active && H[p]->D - t >= MIN_DEPTH) act.push_back(p);
    std::vector<Prob<R>> probs(act.size());
    int nmax = 0, nNmax = 0, mmax = 0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int p = act[a];
      rss_ctx* h = H[p];
      LevelHost& cur = W[p].cur;
      const int d = cur.d, nb = cur.nb, nbox = nb * nb;
      DepthRecords dr;
      dr.d = d;
      dr.nb = nb;
      std::vector<int64_t> oT(nbox), oXi(nbox), oXSNR(nbox), oY(nbox), oS(nbox), oR(nbox), oN(nbox);
      int64_t F = 0, G = 0;
      for (int b = 0; b < nbox; ++b) {
        const int n = cur.n0[b];
        int nN0 = 0;
        for (int x : ring(nb, b, 1)) nN0 += cur.n0[x];
        const int64_t tt = (int64_t)n * n;
        oT[b] = F;
        F += (tt + 3) / 4 + n;
        oXi[b] = F;
        F += tt;
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
      dr.d_F = h->arena.alloc((size_t)F * E);
      dr.d_G = (int*)h->arena.alloc((size_t)G * sizeof(int));
      // per-problem phase lists (kept for the solve); four colours: a
      // colour's boxes ordered by their pass of the Schur update
      for (int c = 0; c < 9; ++c) {
        PhaseHost& P = dr.ph[c];
        for (int q = 0; q < 4; ++q)
          for (int b = 0; b < nbox; ++b)
            if (box_colour(b, nb, h->opt.colours) == c && cur.n0[b] > 0 &&
                (h->opt.colours == 9 ? q == 0 : schur_pass(b, nb) == q))
              P.boxes.push_back(b);
      }
      h->recs.push_back(std::move(dr));
      {
        // ranks (zeroed; k, r, nN adjacent for one readback), offsets and phase
        // lists of this depth in one upload
        DepthRecords& rd = h->recs.back();
        Packer pk;
        pk.zeros(rd.d_k, nbox);
        pk.zeros(rd.d_r, nbox);
        pk.zeros(rd.d_nN, nbox);
        pk.add(rd.d_oT, oT);
        pk.add(rd.d_oXi, oXi);
        pk.add(rd.d_oXSNR, oXSNR);
        pk.add(rd.d_oY, oY);
        pk.add(rd.d_oS, oS);
        pk.add(rd.d_oR, oR);
        pk.add(rd.d_oN, oN);
        for (int c = 0; c < 9; ++c) {
          PhaseHost& P = rd.ph[c];
          pk.add(P.d_box, P.boxes);
          pk.zeros(P.d_prob, P.boxes.size());
        }
        pk.flush(h->arena, s);
      }
      Prob<R>& pr = probs[a];
      pr.L = dev_level<R>(cur, h->x0, h->y0, h->s0);
      pr.rec = dev_records<R>(h->recs.back());
      pr.kp = h->kp;
      pr.P = h->d_P;
      pr.tol = h->tol;
      pr.n_proxy = h->opt.n_proxy;
      pr.proxy_radius = h->opt.proxy_radius;
      nmax = std::max(nmax, cur.nmax);
      nNmax = std::max(nNmax, cur.nNmax);
      mmax = std::max(mmax, 2 * cur.msum_max + 2 * h->opt.n_proxy);
    }
    Prob<R>* d_probs = nullptr;
    Packer pk;  // problem descriptors and merged phase lists of this height: one upload
    pk.add(d_probs, probs);
    // merged colour phases over all active problems, and one shared workspace
    struct Merged {
      std::vector<int> box, prob;
      std::vector<int64_t> oC, oX, oZ, oI, oD;
      std::vector<int64_t> oP, oG, oR;  // Gram ID workspace per slot (doubles)
      int64_t tot = 0, itot = 0, dtot = 0, gtot = 0;
      int rows_ub = 0;                   // most rows of Y = [A_MB; K(proxy, B)] of a slot
      int chunks = 1, chunk_rows = 1;
      int nmax = 0;                      // largest box of the phase
      bool tune = false;                 // time the Gram chunkings (workspace for the largest)
      GramTuneKey key{};
      int pass_lo[5] = {0, 0, 0, 0, 0};  // four colours: slots of Schur pass q are [pass_lo[q], pass_lo[q+1])
    } M[9];
    const int colours = H[0]->opt.colours;
    if (sparsify_min_lds(nmax) > SPARSIFY_LDS_CAP)
      fail(RSS_EUNSUPPORTED, "boxes of " + std::to_string(nmax) + " active points exceed the sparsification's LDS");
    // the ID through the double-double Gram matrix for boxes of up to
    // GRAM_NMAX points, else column-pivoted Householder QR on C
    const bool use_gram = nmax <= gram_nmax();
    int64_t Wmax = 0, Imax = 0, Dmax = 0, Gmax_ws = 0;
    int maxph = 0;
    for (int c = 0; c < 9; ++c) {
      Merged& G = M[c];
      int64_t C = 0, X = 0, Z = 0, I = 0;
      std::vector<int64_t> cx_, xx_, zx_;
      // slots problem by problem (nine colours), or pass by pass and then
      // problem by problem (four colours)
      std::vector<std::pair<int, int>> slots;  // (a, b)
      for (int q = 0; q < (colours == 4 ? 4 : 1); ++q) {
        G.pass_lo[q] = (int)slots.size();
        for (size_t a = 0; a < act.size(); ++a)
          for (int b : H[act[a]]->recs.back().ph[c].boxes)
            if (colours != 4 || schur_pass(b, W[act[a]].cur.nb) == q) slots.push_back({(int)a, b});
      }
      for (int q = (colours == 4 ? 4 : 1); q < 5; ++q) G.pass_lo[q] = (int)slots.size();
      for (const auto& sl : slots) {
        const size_t a = (size_t)sl.first;
        const int b = sl.second;
        const int p = act[a];
        const LevelHost& cur = W[p].cur;
        const int nb = cur.nb;
        {
          const int n = cur.n0[b];
          int msum = 0, nN0 = 0;
          for (int x : ring(nb, b, 2)) msum += cur.n0[x];
          for (int x : ring(nb, b, 1)) nN0 += cur.n0[x];
          const int m = 2 * msum + 2 * H[p]->opt.n_proxy;
          G.rows_ub = std::max(G.rows_ub, msum + H[p]->opt.n_proxy);
          G.nmax = std::max(G.nmax, n);
          G.box.push_back(b);
          G.prob.push_back((int)a);
          cx_.push_back(C);
          if (!use_gram) C += (int64_t)m * n;
          xx_.push_back(X);
          X += (int64_t)n * n;
          zx_.push_back(Z);
          Z += (int64_t)n * (n + nN0);
          G.oI.push_back(I);
          I += 3 * n;
          G.oD.push_back(G.dtot);
          G.dtot += (int64_t)n * n;
        }
      }
      for (size_t i = 0; i < G.box.size(); ++i) {
        G.oC.push_back(cx_[i]);
        G.oX.push_back(C + xx_[i]);
        G.oZ.push_back(C + X + zx_[i]);
      }
      G.tot = C + X + Z;
      G.itot = I;
      if (use_gram && !G.box.empty()) {
        // row chunks per box: the tuned choice of this bucket, else ~2048
        // workgroups; a bucket not tuned yet gets workspace for the most chunks
        const int nslot = (int)G.box.size();
        G.key = gram_tune_key((int)sizeof(R), G.nmax, nslot, G.rows_ub);
        int target = GRAM_TUNE_DEFAULT;
        bool cached = false;
        {
          std::lock_guard<std::mutex> lk(g_gram_tune_mu);
          auto it = g_gram_tune.find(G.key);
          if (it != g_gram_tune.end()) {
            target = it->second.target;
            cached = true;
          }
        }
        G.tune = !cached && gram_tuning_on();
        gram_chunking(G.tune ? GRAM_TUNE_TARGETS[4] : target, nslot, G.nmax, G.rows_ub, G.chunks, G.chunk_rows);
        int64_t o = 0;
        for (size_t i = 0; i < G.box.size(); ++i) {
          const int n = W[act[G.prob[i]]].cur.n0[G.box[i]];
          const int64_t nn = (int64_t)n * n;
          G.oG.push_back(o);
          o += 2 * nn;
          G.oR.push_back(o);
          o += 2 * nn;  // rows of R: high and low parts
          G.oP.push_back(o);
          if (G.chunks > 1) o += (int64_t)G.chunks * 2 * nn;
        }
        G.gtot = o;
        Gmax_ws = std::max(Gmax_ws, o);
      }
      Wmax = std::max(Wmax, G.tot);
      Imax = std::max(Imax, I);
      Dmax = std::max(Dmax, G.dtot);
      maxph = std::max(maxph, (int)G.box.size());
    }
    void* Wd = scr.alloc((size_t)Wmax * E);
    int* Wi = (int*)scr.alloc((size_t)Imax * sizeof(int));
    // FP64 work for the redundant-block inverses too large for LDS
    cx<double>* Wdd = (cx<double>*)scr.alloc((size_t)std::max<int64_t>(1, Dmax) * sizeof(cx<double>));
    double* Wg = use_gram ? (double*)scr.alloc((size_t)std::max<int64_t>(1, Gmax_ws) * sizeof(double)) : nullptr;
    // multi-workgroup ID for colours with few boxes: G workgroups per box
    int Gc[9], Gmax = 1;
    for (int c = 0; c < 9; ++c) {
      Gc[c] = (M[c].box.empty() || H[0]->no_mg) ? 1 : cpqr_mg_groups<R>((int)M[c].box.size(), nmax, mmax);
      Gmax = std::max(Gmax, Gc[c] * (int)M[c].box.size());
    }
    double* pnorm = (double*)scr.alloc((size_t)Gmax * nmax * sizeof(double));
    double* pdot = (double*)scr.alloc((size_t)Gmax * nmax * 2 * sizeof(double));
    unsigned* bars = (unsigned*)scr.alloc((size_t)std::max(1, maxph) * sizeof(unsigned));
    // row counts of the ID matrices, one slice per colour, read back once per height
    int* mrow = (int*)scr.alloc((size_t)9 * std::max(1, maxph) * sizeof(int));
    GemmDesc<R>* desc = (GemmDesc<R>*)scr.alloc((size_t)std::max(1, maxph) * sizeof(GemmDesc<R>));
    const int chunks = (mmax + 63) / 64;
    Phase<R> phs[9];
    GramWs gws[9];
    for (int c = 0; c < 9; ++c) {
      Merged& G = M[c];
      if (G.box.empty()) continue;
      Phase<R>& ph = phs[c];
      ph.nbox = (int)G.box.size();
      pk.add(ph.box, G.box);
      pk.add(ph.prob, G.prob);
      pk.add(ph.oC, G.oC);
      pk.add(ph.oX, G.oX);
      pk.add(ph.oZ, G.oZ);
      pk.add(ph.oI, G.oI);
      pk.add(ph.oD, G.oD);
      ph.mrow = mrow + (size_t)c * std::max(1, maxph);
      ph.W = (cx<R>*)Wd;
      ph.Wi = Wi;
      ph.Wd = Wdd;
      if (use_gram) {
        GramWs& gw = gws[c];
        gw.part = gw.G = gw.Rw = Wg;
        pk.add(gw.oP, G.oP);
        pk.add(gw.oG, G.oG);
        pk.add(gw.oR, G.oR);
        gw.chunks = G.chunks;
        gw.chunk_rows = G.chunk_rows;
      }
    }
    pk.flush(scr, s);
    // the Gram chunking of a bucket met for the first time: each candidate
    // once to warm up and twice timed, then the fastest is kept (and set in gw)
    auto tune_gram = [&](const Phase<R>& ph, GramWs& gw, Merged& G) {
      {
        std::lock_guard<std::mutex> lk(g_gram_tune_mu);
        auto it = g_gram_tune.find(G.key);
        if (it != g_gram_tune.end()) {  // tuned by an earlier phase of this height
          gram_chunking(it->second.target, ph.nbox, G.nmax, G.rows_ub, gw.chunks, gw.chunk_rows);
          return;
        }
      }
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      GramTuneVal best{GRAM_TUNE_DEFAULT, 0, 0.0f};
      int last_chunks = -1;
      for (int target : GRAM_TUNE_TARGETS) {
        int ch = 0, cr = 0;
        gram_chunking(target, ph.nbox, G.nmax, G.rows_ub, ch, cr);
        if (ch == last_chunks) continue;  // the same launch as the previous target
        last_chunks = ch;
        gw.chunks = ch;
        gw.chunk_rows = cr;
        launch_gram<R>(d_probs, ph, gw, G.nmax, s);
        HIPCHK(hipEventRecord(e0, s));
        for (int rep = 0; rep < 2; ++rep) launch_gram<R>(d_probs, ph, gw, G.nmax, s);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const float us = ms * 500.0f;
        if (best.chunks == 0 || us < best.us) best = {target, ch, us};
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      gram_chunking(best.target, ph.nbox, G.nmax, G.rows_ub, gw.chunks, gw.chunk_rows);
      std::lock_guard<std::mutex> lk(g_gram_tune_mu);
      g_gram_tune.emplace(G.key, best);
    };
    for (int c = 0; c < 9; ++c) {
      if (M[c].box.empty()) continue;
      const Phase<R>& ph = phs[c];
      if (use_gram && M[c].tune) tune_gram(ph, gws[c], M[c]);
      if (use_gram) {
        prof.run(RSS_K_ID, s, [&] {
          launch_gram<R>(d_probs, ph, gws[c], M[c].nmax, s);
          launch_chol<R>(d_probs, ph, gws[c], M[c].nmax, s);
        });
      } else {
        prof.run(RSS_K_BUILD_C, s, [&] { launch_build_C<R>(d_probs, ph, chunks, s); });
        prof.run(RSS_K_ID, s, [&] {
          if (Gc[c] < 2 ||
              !launch_cpqr_mg<R>(d_probs, ph, nmax, mmax, Gc[c], pnorm, pdot, bars, d_err, mg_spin_limit(), s))
            launch_cpqr<R>(d_probs, ph, nmax, mmax, s);
        });
      }
      prof.run(RSS_K_SPARSIFY, s, [&] { launch_sparsify<R>(d_probs, ph, nmax, use_gram, s); });
      prof.run(RSS_K_INVERSE, s, [&] { launch_inverse<R>(d_probs, ph, d_err, nmax, s); });
      launch_plan_y<R>(d_probs, ph, desc, s);
      prof.run(RSS_K_GEMM_Y, s, [&] { launch_gemm<R>(desc, ph.nbox, nmax, nmax + nNmax, s); });
      prof.run(RSS_K_COMPACT, s, [&] { launch_compact<R>(d_probs, ph, colours, s); });
      prof.run(RSS_K_SCHUR, s, [&] {
        if (colours != 4) {
          launch_schur<R>(d_probs, ph, nmax + nNmax, s);
          return;
        }
        // four ordered passes: boxes of a pass are 4 apart (no common target block)
        for (int q = 0; q < 4; ++q) {
          const int lo = M[c].pass_lo[q], hi = M[c].pass_lo[q + 1];
          if (hi <= lo) continue;
          Phase<R> sub = ph;
          sub.nbox = hi - lo;
          sub.box += lo;
          sub.prob += lo;
          launch_schur<R>(d_probs, sub, nmax + nNmax, s);
        }
      });
    }
    std::vector<int> mrow_h((size_t)9 * std::max(1, maxph));
    HIPCHK(hipMemcpyAsync(mrow_h.data(), mrow, mrow_h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    // read back ranks and surviving ids of every active problem
    std::vector<std::vector<int>> curk(act.size()), ids(act.size());
    for (size_t a = 0; a < act.size(); ++a) {
      const int p = act[a];
      DepthRecords& dr = H[p]->recs.back();
      const LevelHost& cur = W[p].cur;
      const int nbox = cur.nb * cur.nb;
      dr.k.resize(nbox);
      dr.r.resize(nbox);
      dr.nN.resize(nbox);
      dr.m.assign(nbox, 0);
      curk[a].resize(nbox);
      ids[a].resize(cur.idx.size());
    }
    // two copies per problem (k .. nN and cur .. idx are adjacent) into pinned memory
    std::vector<size_t> rb_off(2 * act.size() + 1, 0);
    for (size_t a = 0; a < act.size(); ++a) {
      const DepthRecords& dr = H[act[a]]->recs.back();
      const LevelHost& cur = W[act[a]].cur;
      rb_off[2 * a + 1] = rb_off[2 * a] + (size_t)((char*)(dr.d_nN + dr.k.size()) - (char*)dr.d_k);
      rb_off[2 * a + 2] = rb_off[2 * a + 1] + (size_t)((char*)(cur.d_idx + cur.idx.size()) - (char*)cur.d_cur);
    }
    char* rb = (char*)pinned.get(rb_off.back());
    for (size_t a = 0; a < act.size(); ++a) {
      const DepthRecords& dr = H[act[a]]->recs.back();
      const LevelHost& cur = W[act[a]].cur;
      HIPCHK(hipMemcpyAsync(rb + rb_off[2 * a], dr.d_k, rb_off[2 * a + 1] - rb_off[2 * a],
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(rb + rb_off[2 * a + 1], cur.d_cur, rb_off[2 * a + 2] - rb_off[2 * a + 1],
                            hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (size_t a = 0; a < act.size(); ++a) {
      DepthRecords& dr = H[act[a]]->recs.back();
      const LevelHost& cur = W[act[a]].cur;
      const size_t nbox = dr.k.size();
      const char* p0 = rb + rb_off[2 * a];
      std::memcpy(dr.k.data(), p0, nbox * sizeof(int));
      std::memcpy(dr.r.data(), p0 + ((char*)dr.d_r - (char*)dr.d_k), nbox * sizeof(int));
      std::memcpy(dr.nN.data(), p0 + ((char*)dr.d_nN - (char*)dr.d_k), nbox * sizeof(int));
      const char* p1 = rb + rb_off[2 * a + 1];
      std::memcpy(curk[a].data(), p1, nbox * sizeof(int));
      if (!ids[a].empty())
        std::memcpy(ids[a].data(), p1 + ((char*)cur.d_idx - (char*)cur.d_cur), ids[a].size() * sizeof(int));
    }
    for (size_t a = 0; a < act.size(); ++a) {
      // the solve sizes its LDS panels by the ranks the level actually has
      DepthRecords& dr = H[act[a]]->recs.back();
      dr.kmax = dr.rmax = dr.qmax = 1;
      for (int v : dr.k) dr.kmax = std::max(dr.kmax, v);
      for (int v : dr.r) dr.rmax = std::max(dr.rmax, v);
      for (size_t b = 0; b < dr.k.size(); ++b) dr.qmax = std::max(dr.qmax, dr.k[b] + dr.nN[b]);
    }
    prof.collect(H[0]->stats.t_class_ms, H[0]->stats.n_class);
    for (int c = 0; c < 9; ++c)
      for (size_t i = 0; i < M[c].box.size(); ++i)
        H[act[M[c].prob[i]]]->recs.back().m[M[c].box[i]] = mrow_h[(size_t)c * std::max(1, maxph) + i];
    scr.clear();

    // ledger, skeleton export, parent lists and transition descriptors
    std::vector<PairDesc> pds;
    std::vector<ListEntry> lists;
    std::vector<Prob<R>> cprobs;      // child levels for the transition launch
    std::vector<int> trans;           // problems that move to a parent level
    int tmr = 0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int p = act[a];
      rss_ctx* h = H[p];
      Work& w = W[p];
      LevelHost& cur = w.cur;
      DepthRecords& dr = h->recs.back();
      const int d = cur.d, nb = cur.nb, nbox = nb * nb;
      const int npx = h->opt.n_proxy;
      std::vector<int> kk(nbox, -1);
      std::vector<int64_t> sid;
      for (int b = 0; b < nbox; ++b) {
        const int n = cur.n0[b];
        if (n == 0) continue;
        const int k = curk[a][b];
        kk[b] = k;
        for (int i = 0; i < k; ++i) sid.push_back(ids[a][cur.ioff[b] + i]);
        const double m = dr.m[b], k_ = dr.k[b], r_ = dr.r[b], nN = dr.nN[b];
        w.flops_id += 4.0 * (4.0 * m * n * k_ - 2.0 * (m + n) * k_ * k_ + 4.0 * k_ * k_ * k_ / 3.0);
        w.kevals += 2.0 * npx * n;
        if (r_ > 0) {
          w.flops_lu += 8.0 / 3.0 * r_ * r_ * r_;
          w.flops_y += 8.0 * r_ * r_ * (k_ + nN);
          w.flops_schur += 8.0 * (k_ + nN) * (k_ + nN) * r_;
          w.fbytes += E * (k_ * r_ + r_ * r_ + 2.0 * (k_ + nN) * r_);
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
      if (d == MIN_DEPTH) {
        std::vector<int> all(nbox);
        for (int b = 0; b < nbox; ++b) all[b] = b;
        w.root_list = sorted_union(all, curk[a], ids[a], cur.ioff);
        continue;  // the level stays alive for the root assembly
      }
      const int pd = d - 1, pnb = 1 << pd, pbox = pnb * pnb;
      std::vector<std::vector<ListEntry>> plist(pbox);
      std::vector<int> pcount(pbox, 0);
      for (int q = 0; q < pbox; ++q) {
        const int px = q % pnb, py = q / pnb;
        std::vector<int> kids;
        for (int j = 0; j < 2; ++j)
          for (int i = 0; i < 2; ++i) kids.push_back((2 * py + j) * nb + (2 * px + i));
        plist[q] = sorted_union(kids, curk[a], ids[a], cur.ioff);
        pcount[q] = (int)plist[q].size();
      }
      LevelHost par;
      par.layout(pd, pcount);
      par.idx.clear();
      std::vector<int64_t> loff(pbox);
      for (int q = 0; q < pbox; ++q) {
        loff[q] = (int64_t)lists.size();
        for (auto& e : plist[q]) {
          par.idx.push_back(e.gid);
          lists.push_back(e);
        }
      }
      alloc_level(h, par, E, s);
      const int pi = (int)cprobs.size();
      Prob<R> cp{};
      cp.L = dev_level<R>(cur, h->x0, h->y0, h->s0);
      cp.kp = h->kp;
      cp.P = h->d_P;
      cprobs.push_back(cp);
      for (int q = 0; q < pbox; ++q)
        for (int sl = 0; sl < 25; ++sl) {
          const int64_t off = par.boff[(size_t)q * 25 + sl];
          if (off < 0) continue;
          const int sdx = sl % 5 - 2, sdy = sl / 5 - 2;
          const int q2 = (q / pnb + sdy) * pnb + (q % pnb + sdx);
          if (pcount[q] == 0 || pcount[q2] == 0) continue;
          // parent boxes 2 apart: every pair of their children is at least 3
          // apart, so no entry comes from a stored child block and the block
          // is the transpose of its mirror bit for bit; the pair with
          // (dy, dx) > (0, 0) writes both, its mirror gets no descriptor
          const bool fresh = std::max(std::abs(sdx), std::abs(sdy)) == 2;
          const bool later = sdy > 0 || (sdy == 0 && sdx > 0);
          PairDesc pd_;
          pd_.dst = (char*)par.d_A + off * E;
          pd_.dstT = nullptr;
          pd_.ldT = 0;
          if (fresh && later) {
            pd_.dstT = (char*)par.d_A + par.boff[(size_t)q2 * 25 + (2 - sdy) * 5 + (2 - sdx)] * E;
            pd_.ldT = pcount[q2];
          }
          pd_.ld = pcount[q];
          pd_.nr = pcount[q];
          pd_.nc = pcount[q2];
          pd_.prob = pi;
          pd_.have_child = 1;
          pd_.roff = loff[q];
          pd_.coff = loff[q2];
          if (!fresh || later) pds.push_back(pd_);
          const int qx = q % pnb, qy = q / pnb, rx = q2 % pnb, ry = q2 / pnb;
          for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) {
              const int ca = (2 * qy + u / 2) * nb + 2 * qx + u % 2;
              const int cb = (2 * ry + v / 2) * nb + 2 * rx + v % 2;
              if (chebyshev(nb, ca, cb) > 2) w.kevals += (double)curk[a][ca] * curk[a][cb];
            }
        }
      tmr = std::max(tmr, par.nmax);
      trans.push_back(p);
      // the parent becomes the current level; the child is freed after the launch
      std::swap(w.cur, par);
      h->tmp_levels.push_back(std::move(par));
    }
    if (!pds.empty()) {
      PairDesc* d_pds = scr.up(pds, s);
      ListEntry* d_lists = scr.up(lists, s);
      Prob<R>* d_cp = scr.up(cprobs, s);
      prof.run(RSS_K_ASSEMBLE, s, [&] {
        launch_assemble_pairs<R>(d_pds, (int)pds.size(), d_lists, tmr, tmr, d_cp, s);
      });
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      scr.clear();
    }
    for (int p : trans) {
      for (auto& L : H[p]->tmp_levels) free_level(H[p], L);
      H[p]->tmp_levels.clear();
    }
  }

  // roots: every remaining index, dense (the top of Alg. a:fact); one batch
  {
    std::vector<PairDesc> pds;
    std::vector<ListEntry> lists;
    std::vector<Prob<R>> cprobs;
    std::vector<RootDesc<R>> rds;
    // complex64 form: the root is inverted in FP64 (A64/tmp64) and rounded into A
    std::vector<RootDesc<double>> rds64;
    std::vector<cx<R>*> root_out;
    constexpr bool f32 = sizeof(R) != sizeof(double);
    int nrmax = 0;
    for (int p = 0; p < np; ++p) {
      rss_ctx* h = H[p];
      Work& w = W[p];
      const int nr = (int)w.root_list.size();
      h->n_root = nr;
      h->stats.n_root = nr;
      if (nr == 0) continue;
      std::vector<int> rid(nr);
      for (int i = 0; i < nr; ++i) rid[i] = w.root_list[i].gid;
      h->d_root_ids = h->arena.up(rid, s);
      const size_t bytes = (size_t)nr * nr * E;
      RootDesc<R> rd;
      rd.A = (cx<R>*)h->arena.alloc(bytes);
      rd.perm = (int*)scr.alloc((size_t)nr * 2 * sizeof(int));
      rd.n = nr;
      rd.W = nullptr;
      rd.gd = nullptr;
      if (f32) {
        RootDesc<double> r64;
        r64.A = (cx<double>*)scr.alloc((size_t)nr * nr * sizeof(cx<double>));
        r64.tmp = (cx<double>*)scr.alloc((size_t)nr * nr * sizeof(cx<double>));
        r64.W = (cx<double>*)scr.alloc(root_work_elems(nr) * sizeof(cx<double>));
        r64.gd = nullptr;
        r64.perm = rd.perm;
        r64.n = nr;
        rds64.push_back(r64);
        root_out.push_back(rd.A);
        rd.tmp = nullptr;
        h->d_root_inv = rd.A;
        h->root_spare = nullptr;
      } else {
        rd.tmp = (cx<R>*)h->arena.alloc(bytes);
        rd.W = (cx<R>*)scr.alloc(root_work_elems(nr) * sizeof(cx<R>));
        // the inverse ends in tmp
        h->d_root_inv = (void*)rd.tmp;
        h->root_spare = (void*)rd.A;
      }
      rds.push_back(rd);
      Prob<R> cp{};
      const bool have = h->D >= MIN_DEPTH;
      if (have) cp.L = dev_level<R>(w.cur, h->x0, h->y0, h->s0);
      cp.kp = h->kp;
      cp.P = h->d_P;
      const int pi = (int)cprobs.size();
      cprobs.push_back(cp);
      PairDesc q;
      q.dst = rd.A;
      q.dstT = nullptr;
      q.ldT = 0;
      q.ld = nr;
      q.nr = nr;
      q.nc = nr;
      q.prob = pi;
      q.have_child = have ? 1 : 0;
      q.roff = (int64_t)lists.size();
      q.coff = q.roff;
      for (auto& e : w.root_list) lists.push_back(e);
      pds.push_back(q);
      nrmax = std::max(nrmax, nr);
      w.flops_lu += 8.0 * (double)nr * nr * nr;
      w.fbytes += (double)nr * nr * E;
      if (!have) {
        w.kevals += (double)nr * nr;
      } else {
        // fresh kernel blocks of the root: pairs of depth-2 boxes more than 2 apart
        const std::vector<int>& kk = h->skel_k.back();
        const int nb = 1 << MIN_DEPTH;
        for (int a = 0; a < nb * nb; ++a)
          for (int b = 0; b < nb * nb; ++b)
            if (kk[a] > 0 && kk[b] > 0 && chebyshev(nb, a, b) > 2) w.kevals += (double)kk[a] * kk[b];
      }
    }
    if (!pds.empty()) {
      PairDesc* d_pds = scr.up(pds, s);
      ListEntry* d_lists = scr.up(lists, s);
      Prob<R>* d_cp = scr.up(cprobs, s);
      // one update-product descriptor per problem, rewritten by every panel
      GemmDesc<R>* gdR = (GemmDesc<R>*)scr.alloc(rds.size() * sizeof(GemmDesc<R>));
      GemmDesc<double>* gd64 = (GemmDesc<double>*)scr.alloc(rds64.size() * sizeof(GemmDesc<double>));
      for (size_t i = 0; i < rds.size(); ++i) rds[i].gd = gdR + i;
      for (size_t i = 0; i < rds64.size(); ++i) rds64[i].gd = gd64 + i;
      RootDesc<R>* d_rd = scr.up(rds, s);
      prof.run(RSS_K_ASSEMBLE, s, [&] {
        launch_assemble_pairs<R>(d_pds, (int)pds.size(), d_lists, nrmax, nrmax, d_cp, s);
      });
      prof.run(RSS_K_ROOT, s, [&] {
        if (f32) {
          for (size_t i = 0; i < rds64.size(); ++i) {
            const int64_t nn = (int64_t)rds64[i].n * rds64[i].n;
            HIPCHK(hipMemsetAsync(rds64[i].A, 0, (size_t)nn * sizeof(cx<double>), s));
            launch_axpy_from_c64((const cx<float>*)rds[i].A, nn, 1, nullptr, rds64[i].A, s);
          }
          RootDesc<double>* d_rd64 = scr.up(rds64, s);
          launch_root_inverse<double>(d_rd64, (int)rds64.size(), nrmax, gd64, d_err, s);
          for (size_t i = 0; i < rds64.size(); ++i) {
            const int nn = rds64[i].n;
            launch_cast_c64(rds64[i].tmp, (int64_t)nn * nn, 1, (cx<float>*)root_out[i], s);
          }
        } else {
          launch_root_inverse<R>(d_rd, (int)rds.size(), nrmax, gdR, d_err, s);
        }
      });
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    }
    scr.clear();
    for (int p = 0; p < np; ++p) {
      rss_ctx* h = H[p];
      if (h->root_spare) {
        h->arena.release(h->root_spare);
        h->root_spare = nullptr;
      }
      if (W[p].active) free_level(h, W[p].cur);
    }
  }
  HIPCHK(hipEventRecord(ev1, s));
  HIPCHK(hipEventSynchronize(ev1));
  prof.collect(H[0]->stats.t_class_ms, H[0]->stats.n_class);
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // a barrier timeout first: the boxes behind it were not factored, so a zero
  // pivot found after it proves nothing (the factorization is redone)
  if (err & ERRF_TIMEOUT) throw MgTimeout{};
  if (err & ERRF_SINGULAR) fail(RSS_ESINGULAR, "zero pivot in a redundant-block or root inverse");
  for (int p = 0; p < np; ++p) {
    rss_ctx* h = H[p];
    Work& w = W[p];
    h->stats.t_factor_ms = ms;
    h->stats.flops_id = w.flops_id;
    h->stats.flops_lu = w.flops_lu;
    h->stats.flops_y = w.flops_y;
    h->stats.flops_schur = w.flops_schur;
    h->stats.factor_bytes = w.fbytes;
    h->stats.kernel_evals = w.kevals;
    h->stats.device_bytes = h->arena.bytes;
  }
}

// The launches of one batched apply (the solve sweeps of Sec. 2.6: forward over the
// records in factor order, the root, backward in reverse), with every
// descriptor they read in device memory.  The vectors z_p are reached only
// through the descriptor tables (SolveProb::z, RootApply::z), so a plan can be
// replayed on other vectors of the same shape after set_z rewrites them.
template <class R>
struct ApplyPlan {
  struct HPhase {
    SolveProb<R>* d_sp = nullptr;
    std::vector<SolveProb<R>> sp;  // host copy (z rewritten per call)
    std::vector<int> owner;        // problem of each entry of sp
    Phase<R> ph[9];
    int kmax = 0, rmax = 0, qmax = 0;
    int gmax = 0;                  // largest valid ncg (LDS budget)
    SolveTile tile[9];             // per colour phase
  };
  std::vector<HPhase> HP;
  int tmax = -1, nrhs_max = 0, nmax = 0;
  cx<R>* Wk = nullptr;
  size_t wcap = 0;                 // entries of Wk
  RootApply<R>* d_ra = nullptr;
  std::vector<RootApply<R>> ra;
  std::vector<int> ra_owner;
  GemmDesc<R>* desc = nullptr;

  void build(const std::vector<rss_ctx*>& H, const std::vector<cx<R>*>& Z, const std::vector<int>& nrhs,
             Scratch& mem, hipStream_t s) {
    const int np = (int)H.size();
    for (int p = 0; p < np; ++p) {
      tmax = std::max(tmax, (int)H[p]->recs.size() - 1);
      nrhs_max = std::max(nrhs_max, nrhs[p]);
    }
    // per height: SolveProb array over the problems that have that height, and merged phases
    HP.assign(tmax + 1, HPhase{});
    for (int t = 0; t <= tmax; ++t) {
      std::vector<int> idxmap(np, -1);
      for (int p = 0; p < np; ++p)
        if (t < (int)H[p]->recs.size()) {
          idxmap[p] = (int)HP[t].sp.size();
          SolveProb<R> q;
          q.rec = dev_records<R>(H[p]->recs[t]);
          q.z = Z[p];
          q.ldz = H[p]->N;
          q.nrhs = nrhs[p];
          HP[t].sp.push_back(q);
          HP[t].owner.push_back(p);
          HP[t].kmax = std::max(HP[t].kmax, H[p]->recs[t].kmax);
          HP[t].rmax = std::max(HP[t].rmax, H[p]->recs[t].rmax);
          HP[t].qmax = std::max(HP[t].qmax, H[p]->recs[t].qmax);
        }
      HP[t].d_sp = mem.up(HP[t].sp, s);
      for (int c = 0; c < 9; ++c) {
        Phase<R>& ph = HP[t].ph[c];
        ph = Phase<R>{};
        if (HP[t].sp.size() == 1) {
          const PhaseHost& P = H[HP[t].owner[0]]->recs[t].ph[c];
          ph.nbox = (int)P.boxes.size();
          ph.box = P.d_box;
          ph.prob = P.d_prob;
        } else {
          std::vector<int> box, prob;
          for (int p = 0; p < np; ++p)
            if (idxmap[p] >= 0)
              for (int b : H[p]->recs[t].ph[c].boxes) {
                box.push_back(b);
                prob.push_back(idxmap[p]);
              }
          ph.nbox = (int)box.size();
          if (ph.nbox) {
            ph.box = mem.up(box, s);
            ph.prob = mem.up(prob, s);
          }
        }
        for (int p = 0; p < np; ++p)
          if (idxmap[p] >= 0 && H[p]->opt.colours == 4) ph.atomic_nbr = 1;
      }
    }
    // tiles: the tuned choice for the level's shape, else the defaults; the
    // work buffer is sized for the largest slice count a tile may take
    size_t wel = 1;
    for (int t = 0; t <= tmax; ++t) {
      HP[t].gmax = solve_group<R>(HP[t].kmax, HP[t].rmax, nrhs_max);
      if (HP[t].gmax == 0) fail(RSS_EUNSUPPORTED, "ranks too large for the solve's LDS panels");
      apply_choice(t, tuned_choice(tune_key(t)));
      for (int c = 0; c < 9; ++c)
        if (HP[t].ph[c].nbox)
          wel = std::max(wel, solve_work_elems<R>(HP[t].ph[c].nbox, HP[t].rmax, max_slices(t, c), nrhs_max));
    }
    // partial products between the two launches of each sweep step
    wcap = wel;
    Wk = (cx<R>*)mem.alloc(wel * sizeof(cx<R>));
    for (int p = 0; p < np; ++p) {
      const int nr = H[p]->n_root;
      if (nr == 0) continue;
      RootApply<R> q;
      q.Ainv = (const cx<R>*)H[p]->d_root_inv;
      q.ids = H[p]->d_root_ids;
      q.n = nr;
      q.z = Z[p];
      q.ldz = H[p]->N;
      q.nrhs = nrhs[p];
      q.ws = (cx<R>*)mem.alloc((size_t)nr * nrhs[p] * 2 * sizeof(cx<R>));
      ra.push_back(q);
      ra_owner.push_back(p);
      nmax = std::max(nmax, nr);
    }
    if (!ra.empty()) {
      d_ra = mem.up(ra, s);
      desc = (GemmDesc<R>*)mem.alloc(ra.size() * sizeof(GemmDesc<R>));
    }
  }

  // Tile choice of a level: the RHS group width as a divisor of the largest
  // valid one (1, 2 or 4) and the slice count as a multiple of the default
  // (x1/2, x1 or x2, clamped to 1 .. SOLVE_SMAX).
  struct Choice {
    int gdiv = 1, smul = 2;  // smul: 1 = half, 2 = default, 4 = double
    bool fused = false;      // each sweep step in one launch (one workgroup per box)
  };
  static constexpr int NGDIV = 3, NSMUL = 3;
  static int gdiv_of(int i) { return 1 << i; }
  static int smul_of(int i) { return 1 << i; }
  int slices(int t, int c, int smul) const {
    const int S0 = solve_slices(HP[t].ph[c].nbox, HP[t].qmax);
    return std::max(1, std::min(SOLVE_SMAX, S0 * smul / 2));
  }
  int max_slices(int t, int c) const { return slices(t, c, smul_of(NSMUL - 1)); }
  bool fused_ok(int t, Choice ch) const {
    return solve_fused_fits<R>(HP[t].kmax, HP[t].rmax, std::max(1, HP[t].gmax / ch.gdiv));
  }
  void apply_choice(int t, Choice ch) {
    const int ncg = std::max(1, HP[t].gmax / ch.gdiv);
    const bool fused = ch.fused && fused_ok(t, ch);
    for (int c = 0; c < 9; ++c) HP[t].tile[c] = SolveTile{ncg, fused ? 1 : slices(t, c, ch.smul), fused};
  }
  // the level's shape as a tuning key: precision, largest valid group width
  // and box count rounded up to powers of two, the ranks rounded up to 8
  std::array<int, 6> tune_key(int t) const {
    auto pow2 = [](int v) {
      int p = 1;
      while (p < v) p <<= 1;
      return p;
    };
    int nb = 0;
    for (int c = 0; c < 9; ++c) nb += HP[t].ph[c].nbox;
    return {(int)sizeof(R), pow2(HP[t].gmax), (HP[t].kmax + 7) / 8, (HP[t].rmax + 7) / 8,
            (HP[t].qmax + 31) / 32, pow2(nb)};
  }

  // Measure the tile choices of every level on this plan's shapes (vectors
  // of zeros, so the caller's data is untouched) and record the fastest: per
  // level, first the group width at the default slice count, then the slice
  // count at that width, then the fused kernels at that width, each timed as
  // one whole apply after a warm-up.  Levels
  // whose key is already tuned keep their choice.
  void autotune(const std::vector<int64_t>& N, const std::vector<int>& nrhs, Scratch& mem, hipStream_t s) {
    std::vector<int> todo;
    for (int t = 0; t <= tmax; ++t)
      if (!tuned_lookup(tune_key(t), nullptr)) todo.push_back(t);
    if (todo.empty()) return;
    std::vector<cx<R>*> Zt;
    for (size_t p = 0; p < N.size(); ++p) {
      const size_t bytes = (size_t)N[p] * nrhs[p] * sizeof(cx<R>);
      cx<R>* z = (cx<R>*)mem.alloc(bytes);
      HIPCHK(hipMemsetAsync(z, 0, bytes, s));
      Zt.push_back(z);
    }
    std::vector<cx<R>*> Zsave = current_z();
    set_z(Zt, s);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_apply = [&]() {
      HIPCHK(hipEventRecord(e0, s));
      launch(s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    launch(s);  // warm-up
    for (int t : todo) {
      Choice best;
      float tb = 1e30f;
      for (int gi = 0; gi < NGDIV; ++gi) {
        Choice ch;
        ch.gdiv = gdiv_of(gi);
        if (gi > 0 && HP[t].gmax / ch.gdiv < 1) break;
        apply_choice(t, ch);
        const float ms = time_apply();
        if (ms < tb) tb = ms, best = ch;
      }
      for (int si = 0; si < NSMUL; ++si) {
        Choice ch = best;
        ch.smul = smul_of(si);
        if (ch.smul == 2) continue;  // the default, timed above
        apply_choice(t, ch);
        const float ms = time_apply();
        if (ms < tb) tb = ms, best = ch;
      }
      {
        Choice ch = best;
        ch.fused = true;
        if (fused_ok(t, ch)) {
          apply_choice(t, ch);
          const float ms = time_apply();
          if (ms < tb) tb = ms, best = ch;
        }
      }
      apply_choice(t, best);
      tuned_store(tune_key(t), best);
    }
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    set_z(Zsave, s);
    HIPCHK(hipStreamSynchronize(s));
  }

  void force_fused() {
    for (int t = 0; t <= tmax; ++t) {
      Choice ch;
      ch.fused = true;
      apply_choice(t, ch);
    }
  }

  std::vector<cx<R>*> current_z() const {
    // the vectors as the descriptors hold them, by problem
    int np = 0;
    for (auto& hp : HP)
      for (int o : hp.owner) np = std::max(np, o + 1);
    for (int o : ra_owner) np = std::max(np, o + 1);
    std::vector<cx<R>*> Z(np, nullptr);
    for (auto& hp : HP)
      for (size_t e = 0; e < hp.sp.size(); ++e) Z[hp.owner[e]] = hp.sp[e].z;
    for (size_t e = 0; e < ra.size(); ++e) Z[ra_owner[e]] = ra[e].z;
    return Z;
  }

  // process-wide table of tuned choices (shared by all handles and servers)
  static std::mutex& tuned_mu() {
    static std::mutex m;
    return m;
  }
  static std::map<std::array<int, 6>, Choice>& tuned_table() {
    static std::map<std::array<int, 6>, Choice> m;
    return m;
  }
  static bool tuned_lookup(const std::array<int, 6>& key, Choice* out) {
    std::lock_guard<std::mutex> lk(tuned_mu());
    auto it = tuned_table().find(key);
    if (it == tuned_table().end()) return false;
    if (out) *out = it->second;
    return true;
  }
  static Choice tuned_choice(const std::array<int, 6>& key) {
    Choice ch;
    tuned_lookup(key, &ch);
    return ch;
  }
  static void tuned_store(const std::array<int, 6>& key, Choice ch) {
    std::lock_guard<std::mutex> lk(tuned_mu());
    tuned_table()[key] = ch;
  }

  // point the descriptor tables at new vectors (same shapes as at build)
  void set_z(const std::vector<cx<R>*>& Z, hipStream_t s) {
    for (auto& hp : HP) {
      for (size_t e = 0; e < hp.sp.size(); ++e) hp.sp[e].z = Z[hp.owner[e]];
      HIPCHK(hipMemcpyAsync(hp.d_sp, hp.sp.data(), hp.sp.size() * sizeof(SolveProb<R>),
                            hipMemcpyHostToDevice, s));
    }
    if (!ra.empty()) {
      for (size_t e = 0; e < ra.size(); ++e) ra[e].z = Z[ra_owner[e]];
      HIPCHK(hipMemcpyAsync(d_ra, ra.data(), ra.size() * sizeof(RootApply<R>), hipMemcpyHostToDevice, s));
    }
  }

  // the kernel launches only (no copies, allocations or synchronisation), so
  // that a stream capture records exactly these
  void launch(hipStream_t s) const {
    for (int t = 0; t <= tmax; ++t)
      for (int c = 0; c < 9; ++c)
        launch_solve_fwd<R>(HP[t].d_sp, HP[t].ph[c], nrhs_max, HP[t].kmax, HP[t].rmax, HP[t].qmax,
                            HP[t].tile[c], Wk, s);
    if (!ra.empty()) launch_root_apply<R>(d_ra, (int)ra.size(), nmax, nrhs_max, desc, s);
    for (int t = tmax; t >= 0; --t)
      for (int c = 8; c >= 0; --c)
        launch_solve_bwd<R>(HP[t].d_sp, HP[t].ph[c], nrhs_max, HP[t].kmax, HP[t].rmax, HP[t].qmax,
                            HP[t].tile[c], Wk, s);
  }
};

// An apply plan of one handle captured into a HIP graph: its memory, the
// captured graph and the executable instance, kept in the handle per
// (precision, nrhs) and replayed by every later apply of that shape.
template <class R>
struct ApplyGraph : ApplyGraphBase {
  Scratch mem;
  ApplyPlan<R> plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~ApplyGraph() override {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

std::atomic<bool> g_use_graphs{true};
}  // namespace
namespace rss {
thread_local bool g_server_thread = false;
}
namespace {

template <class R>
void maybe_autotune(ApplyPlan<R>& plan, const std::vector<rss_ctx*>& H, const std::vector<int>& nrhs,
                    hipStream_t s) {
  // the server's merged batches only reuse tuned shapes: their compositions
  // vary, and tuning inside a request stream would land on request latency
  if (g_autotune_mode.load() == 2) {  // every level fused where it fits (no timing)
    plan.force_fused();
    return;
  }
  if (!g_autotune.load() || (H.size() != 1 && g_server_thread)) return;
  std::vector<int64_t> N;
  for (auto* h : H) N.push_back(h->N);
  Scratch tmp;
  plan.autotune(N, nrhs, tmp, s);
}

// z_p <- F_p^{-1} z_p for every handle of a batch (complex<R>, N_p x nrhs_p,
// ld N_p), on stream s: one launch per (height, colour) and direction.  A
// batch of one handle replays that handle's captured graph for this nrhs
// (captured on first use); a batch of several handles launches its merged
// plan directly, and so do the server's threads: HIP rejects frees and other
// calls made on one thread while another thread captures, and the server's
// factor worker runs beside its solve worker.
template <class R>
void apply_batch(const std::vector<rss_ctx*>& H, const std::vector<cx<R>*>& Z,
                 const std::vector<int>& nrhs, hipStream_t s) {
  if (H.size() == 1 && g_use_graphs.load() && !g_server_thread) {
    rss_ctx* h = H[0];
    const std::pair<int, int> key{(int)sizeof(R), nrhs[0]};
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
      if (h->graphs.size() >= rss_ctx::MAX_GRAPHS) {
        // drop the least recently used capture (the stream is idle: every
        // apply ends with a synchronisation)
        auto lru = h->graphs.begin();
        for (auto jt = h->graphs.begin(); jt != h->graphs.end(); ++jt)
          if (jt->second->last_use < lru->second->last_use) lru = jt;
        h->graphs.erase(lru);
      }
      std::unique_ptr<ApplyGraph<R>> g(new ApplyGraph<R>());
      g->plan.build(H, Z, nrhs, g->mem, s);
      maybe_autotune(g->plan, H, nrhs, s);
      HIPCHK(hipStreamSynchronize(s));  // descriptor uploads done before the capture
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      g->plan.launch(s);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(s, &graph);
      g->graph = graph;
      HIPCHK(ec);
      HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
      it = h->graphs.emplace(key, std::move(g)).first;
    }
    ApplyGraph<R>* g = static_cast<ApplyGraph<R>*>(it->second.get());
    g->last_use = ++h->graph_clock;
    g->plan.set_z(Z, s);
    HIPCHK(hipGraphLaunch(g->exec, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));  // the host copies of the descriptors are reused next call
    return;
  }
  Scratch scr;
  ApplyPlan<R> plan;
  plan.build(H, Z, nrhs, scr, s);
  maybe_autotune(plan, H, nrhs, s);
  plan.launch(s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));  // scratch descriptors are freed on return
}

// One refined solve in progress: the refinement of rss_solve
//   x = F^{-1} b, then x += F^{-1} (b - A x) until max_j ||r_j|| / ||b_j|| <= refine_tol
// (at most refine_steps corrections), advanced one step at a time, so that a
// caller (the solve server) can add and retire solves between steps.  Without
// refinement (refine_steps < 0) a job is one application.  The residual comes
// from the handle's grid operator (rss_set_residual_op) or the on-the-fly sum.
struct RefineJob {
  rss_ctx* h = nullptr;
  cx<double>* B = nullptr;  // the caller's right-hand sides, the solution on finish
  int nrhs = 0;
  Scratch mem;
  cx<double>*b = nullptr, *x = nullptr, *r = nullptr;
  cx<double>* xb = nullptr;  // best iterate so far, when it is not the current x
  double* nrm = nullptr;
  cx<float>* z = nullptr;
  std::vector<double> bn, rn;
  double relres = 1.0;
  double best = HUGE_VAL;    // relres of the best iterate
  bool best_is_x = false;    // the best iterate is the current x (else xb)
  bool refine = true;
  int it = 0;
  bool done = false;
};

RefineJob* refine_begin_impl(rss_ctx* h, void* Bv, int nrhs, hipStream_t s) {
  std::unique_ptr<RefineJob> j(new RefineJob());
  j->h = h;
  j->B = (cx<double>*)Bv;
  j->nrhs = nrhs;
  j->refine = h->refine_steps >= 0;
  const size_t tot = (size_t)h->N * nrhs;
  j->b = (cx<double>*)j->mem.alloc(tot * sizeof(cx<double>));
  j->x = (cx<double>*)j->mem.alloc(tot * sizeof(cx<double>));
  j->r = (cx<double>*)j->mem.alloc(tot * sizeof(cx<double>));
  j->nrm = (double*)j->mem.alloc((size_t)nrhs * 2 * sizeof(double));
  j->z = h->precision == RSS_FP32_REFINE ? (cx<float>*)j->mem.alloc(tot * sizeof(cx<float>)) : nullptr;
  HIPCHK(hipMemcpyAsync(j->b, Bv, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(j->x, 0, tot * sizeof(cx<double>), s));
  HIPCHK(hipMemcpyAsync(j->r, Bv, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
  j->bn.resize(nrhs);
  j->rn.resize(nrhs);
  launch_colnorms(j->b, h->N, nrhs, j->nrm + nrhs, s);
  HIPCHK(hipMemcpyAsync(j->bn.data(), j->nrm + nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  h->stats.last_iters = 0;
  return j.release();
}

// one step of every job (same precision): the corrections d = F^{-1} r in
// one batched application, x += d, then r = b - A x (jobs with grid
// operators by FFT, the others in one on-the-fly launch) and the convergence
// test; jobs without refinement end after their application
void refine_step_impl(const std::vector<RefineJob*>& live, hipStream_t s) {
  if (live.empty()) return;
  const bool fp32 = live[0]->h->precision == RSS_FP32_REFINE;
  std::vector<rss_ctx*> LH;
  std::vector<int> Lnr;
  for (auto* j : live) {
    if (j->h->precision != live[0]->h->precision) fail(RSS_EINVAL, "a step must share the precision");
    LH.push_back(j->h);
    Lnr.push_back(j->nrhs);
  }
  if (fp32) {
    std::vector<cx<float>*> Z;
    for (auto* j : live) {
      launch_colnorms(j->r, j->h->N, j->nrhs, j->nrm, s);
      launch_scale_to_c64(j->r, j->h->N, j->nrhs, j->nrm, j->z, s);
      Z.push_back(j->z);
    }
    apply_batch<float>(LH, Z, Lnr, s);
    for (auto* j : live) launch_axpy_from_c64(j->z, j->h->N, j->nrhs, j->nrm, j->x, s);
  } else {
    std::vector<cx<double>*> Z;
    for (auto* j : live) Z.push_back(j->r);
    apply_batch<double>(LH, Z, Lnr, s);
    for (auto* j : live) launch_add_c128(j->x, j->r, (int64_t)j->h->N * j->nrhs, s);
  }
  std::vector<RefineJob*> res;
  for (auto* j : live) {
    if (!j->refine) {
      j->done = true;
      j->best_is_x = true;
      j->relres = -1.0;
    } else {
      res.push_back(j);
    }
  }
  if (res.empty()) return;
  {
    Scratch rscr;
    std::vector<ResProblem> rp;
    for (auto* j : res) {
      rss_ctx* h = j->h;
      if (h->gridop) {
        h->gridop->apply(j->x, j->b, j->r, j->nrhs, 1, s);
        continue;
      }
      if (!h->d_tperm) {
        const std::vector<int> perm = spatial_order(h->h_points.data(), h->N);
        h->d_tperm = h->arena.up(perm, s);
      }
      rp.push_back({h->kp, h->d_P, h->N, j->x, j->b, j->r, j->nrhs, h->d_tperm});
    }
    if (!rp.empty()) residual_batch(rp, rscr, s);
    for (auto* j : res) {
      launch_colnorms(j->r, j->h->N, j->nrhs, j->nrm, s);
      HIPCHK(hipMemcpyAsync(j->rn.data(), j->nrm, j->nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  }
  for (auto* j : res) {
    // the largest column relres; a NaN in any column makes it NaN (never converged)
    j->relres = 0.0;
    for (int c = 0; c < j->nrhs; ++c) {
      const double bnc = j->bn[c], rnc = j->rn[c];
      const double q = (std::isnan(bnc) || std::isnan(rnc)) ? std::numeric_limits<double>::quiet_NaN()
                                                             : (bnc > 0 ? rnc / bnc : 0.0);
      if (std::isnan(q) || std::isnan(j->relres))
        j->relres = std::numeric_limits<double>::quiet_NaN();
      else
        j->relres = std::max(j->relres, q);
    }
    if (j->relres <= j->h->opt.refine_tol || j->it >= j->h->refine_steps) j->done = true;
    // a NaN relres never counts as an improvement
    const bool better = j->relres < j->best;
    if (better) j->best = j->relres;
    if (better && !j->done) {
      // x changes in the next step: keep a copy of this iterate
      const size_t tot = (size_t)j->h->N * j->nrhs;
      if (!j->xb) j->xb = (cx<double>*)j->mem.alloc(tot * sizeof(cx<double>));
      HIPCHK(hipMemcpyAsync(j->xb, j->x, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
    }
    j->best_is_x = better;
    if (!j->done) j->it++;
  }
}

// the best iterate to B and the handle's statistics; RSS_ENOCONV when the
// refinement missed refine_tol
int refine_finish_impl(RefineJob* j, hipStream_t s) {
  const size_t tot = (size_t)j->h->N * j->nrhs;
  // the best iterate: the last one unless refinement stalled or diverged
  const cx<double>* xo = (j->best_is_x || !j->xb) ? j->x : j->xb;
  HIPCHK(hipMemcpyAsync(j->B, xo, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));  // the job's buffers are freed with it
  if (!j->best_is_x && j->xb) j->relres = j->best;
  j->h->stats.last_relres = j->relres;
  j->h->stats.last_iters = j->it;
  if (j->refine && !(j->relres <= j->h->opt.refine_tol)) {
    g_err = "refinement did not reach refine_tol";
    return RSS_ENOCONV;
  }
  return RSS_OK;
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


// validate the arguments and create a handle (no device work beyond the points)
rss_ctx* make_ctx(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
                  const rss_options* opt, const rss_ctx* shared) {
  validate(points, n, k, tol, leaf);
  std::unique_ptr<rss_ctx> h(new rss_ctx());
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
  if (h->opt.precision != RSS_FP64 && h->opt.precision != RSS_FP32_REFINE)
    fail(RSS_EINVAL, "unknown precision");
  if (h->opt.colours == 0) h->opt.colours = 9;
  if (h->opt.colours != 9 && h->opt.colours != 4) fail(RSS_EINVAL, "colours must be 0, 4 or 9");
  // refinement steps after the first solve (-1: no refinement, plain apply)
  if (h->opt.precision == RSS_FP32_REFINE)
    h->refine_steps = h->opt.max_refine == 0 ? 10 : (h->opt.max_refine < 0 ? -1 : h->opt.max_refine);
  else
    h->refine_steps = h->opt.max_refine > 0 ? h->opt.max_refine : -1;
  h->precision = h->opt.precision;
  h->prof.on = h->opt.profile != 0;
  h->stats.precision = h->precision;
  h->stats.n = n;
  h->stats.last_relres = -1.0;
  if (h->opt.stream) {
    h->stream = (hipStream_t)h->opt.stream;
  } else if (shared) {
    h->stream = shared->stream;
    h->stream_owner = shared->stream_owner;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    hipStream_t st = h->stream;
    h->stream_owner = std::shared_ptr<void>((void*)st, [](void* q) {
      (void)hipStreamSynchronize((hipStream_t)q);
      (void)hipStreamDestroy((hipStream_t)q);
    });
  }
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
  h->h_points.assign(points, points + 2 * n);
  h->d_P = (double*)h->arena.alloc((size_t)n * 2 * sizeof(double));
  HIPCHK(hipMemcpyAsync(h->d_P, points, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice,
                        h->stream));
  h->d_err = (int*)h->arena.alloc(sizeof(int));
  HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->stream));
  return h.release();
}

void destroy_ctx(rss_ctx* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  delete h;  // the arena frees device memory; the stream goes with its last handle
}

void factor_handles(std::vector<rss_ctx*>& H) {
  hipStream_t s = H[0]->stream;
  for (size_t p = 1; p < H.size(); ++p)
    if (H[p]->stream != s) HIPCHK(hipStreamSynchronize(H[p]->stream));  // points uploaded
  if (H[0]->precision == RSS_FP64) factor_batch<double>(H, s);
  else factor_batch<float>(H, s);
  for (auto* h : H) h->stats.device_bytes = h->arena.bytes;
}

}  // namespace

// The refinement steps for the solve server (rss_server.cpp): status codes in
// place of exceptions, jobs as opaque pointers.
namespace rss {
int refine_begin(rss_handle h, void* B, int nrhs, void** job) {
  *job = nullptr;
  return run([&] {
    if (!h || !B || nrhs < 1) fail(RSS_EINVAL, "bad solve arguments");
    *job = refine_begin_impl(h, B, nrhs, h->stream);
  });
}
int refine_step(void* const* jobs, int n) {
  if (n < 1) return RSS_OK;
  return run([&] {
    std::vector<RefineJob*> live;
    for (int i = 0; i < n; ++i) live.push_back((RefineJob*)jobs[i]);
    refine_step_impl(live, live[0]->h->stream);
  });
}
bool refine_done(const void* job) { return ((const RefineJob*)job)->done; }
int refine_finish(void* job, double* relres, int* iters) {
  RefineJob* j = (RefineJob*)job;
  int code = RSS_OK;
  const int rc = run([&] { code = refine_finish_impl(j, j->h->stream); });
  if (relres) *relres = j->relres;
  if (iters) *iters = j->it;
  delete j;
  return rc != RSS_OK ? rc : code;
}
void refine_free(void* job) {
  RefineJob* j = (RefineJob*)job;
  if (j && j->h) (void)hipStreamSynchronize(j->h->stream);
  delete j;
}
}  // namespace rss

extern "C" {

int rss_factor_ex(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
                  const rss_options* opt, rss_handle* out) {
  if (out) *out = nullptr;
  rss_ctx* h = nullptr;
  const int rc = run([&] {
    if (!out) fail(RSS_EINVAL, "null output handle pointer");
    for (int attempt = 0;; ++attempt) {
      h = make_ctx(points, n, k, tol, leaf, opt, nullptr);
      h->no_mg = attempt > 0;
      std::vector<rss_ctx*> H{h};
      try {
        factor_handles(H);
        h->stats.id_retries = attempt;
        break;
      } catch (const MgTimeout&) {
        if (attempt > 0) fail(RSS_EHIP, "a per-box device barrier timed out");
        destroy_ctx(h);
        h = nullptr;
      }
    }
  });
  if (rc != RSS_OK) {
    destroy_ctx(h);
    return rc;
  }
  *out = h;
  return RSS_OK;
}

int rss_factor_batch(int nprob, const double* const* points, const int64_t* n,
                     const rss_kernel* kernels, double tol, int leaf, const rss_options* opt,
                     rss_handle* out) {
  std::vector<rss_ctx*> H;
  const int rc = run([&] {
    if (nprob < 1 || !points || !n || !kernels || !out) fail(RSS_EINVAL, "bad batch arguments");
    for (int p = 0; p < nprob; ++p) out[p] = nullptr;
    for (int attempt = 0;; ++attempt) {
      for (int p = 0; p < nprob; ++p) {
        H.push_back(make_ctx(points[p], n[p], &kernels[p], tol, leaf, opt, p ? H[0] : nullptr));
        H.back()->no_mg = attempt > 0;
      }
      try {
        factor_handles(H);
        for (auto* h : H) h->stats.id_retries = attempt;
        break;
      } catch (const MgTimeout&) {
        if (attempt > 0) fail(RSS_EHIP, "a per-box device barrier timed out");
        for (auto it = H.rbegin(); it != H.rend(); ++it) destroy_ctx(*it);
        H.clear();
      }
    }
  });
  if (rc != RSS_OK) {
    for (auto* h : H) destroy_ctx(h);
    return rc;
  }
  for (int p = 0; p < nprob; ++p) out[p] = H[p];
  return RSS_OK;
}

int rss_apply_batch(int nh, rss_handle* hs, void* const* B, const int* nrhs) {
  return run([&] {
    if (nh < 1 || !hs || !B || !nrhs) fail(RSS_EINVAL, "bad batch arguments");
    std::vector<rss_ctx*> H(hs, hs + nh);
    for (int p = 0; p < nh; ++p) {
      if (!H[p] || !B[p] || nrhs[p] < 1) fail(RSS_EINVAL, "bad batch entry");
      if (H[p]->precision != H[0]->precision) fail(RSS_EINVAL, "mixed precisions in a batch");
      if (H[p]->opt.colours != H[0]->opt.colours) fail(RSS_EINVAL, "mixed schedules in a batch");
    }
    hipStream_t s = H[0]->stream;
    for (int p = 1; p < nh; ++p)
      if (H[p]->stream != s) HIPCHK(hipStreamSynchronize(H[p]->stream));
    std::vector<int> nr(nrhs, nrhs + nh);
    if (H[0]->precision == RSS_FP64) {
      std::vector<cx<double>*> Z;
      for (int p = 0; p < nh; ++p) Z.push_back((cx<double>*)B[p]);
      apply_batch<double>(H, Z, nr, s);
    } else {
      Scratch scr;
      std::vector<cx<float>*> Z;
      for (int p = 0; p < nh; ++p) {
        const size_t tot = (size_t)H[p]->N * nr[p];
        cx<float>* z = (cx<float>*)scr.alloc(tot * sizeof(cx<float>));
        launch_cast_c64((const cx<double>*)B[p], H[p]->N, nr[p], z, s);
        HIPCHK(hipMemsetAsync(B[p], 0, tot * sizeof(cx<double>), s));
        Z.push_back(z);
      }
      apply_batch<float>(H, Z, nr, s);
      for (int p = 0; p < nh; ++p)
        launch_axpy_from_c64(Z[p], H[p]->N, nr[p], nullptr, (cx<double>*)B[p], s);
      HIPCHK(hipStreamSynchronize(s));
    }
  });
}

int rss_factor(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
               rss_handle* out) {
  return rss_factor_ex(points, n, k, tol, leaf, nullptr, out);
}

int rss_apply(rss_handle h, void* B, int nrhs) { return rss_apply_batch(1, &h, &B, &nrhs); }

int rss_solve_batch(int nh, rss_handle* hs, void* const* B, const int* nrhs) {
  int code = RSS_OK;
  const int rc = run([&] {
    if (nh < 1 || !hs || !B || !nrhs) fail(RSS_EINVAL, "bad batch arguments");
    std::vector<rss_ctx*> H(hs, hs + nh);
    for (int p = 0; p < nh; ++p) {
      if (!H[p] || !B[p]) fail(RSS_EINVAL, "null argument");
      if (nrhs[p] < 1) fail(RSS_EINVAL, "nrhs must be >= 1");
      if (H[p]->precision != H[0]->precision || (H[p]->refine_steps >= 0) != (H[0]->refine_steps >= 0))
        fail(RSS_EINVAL, "a batch must share precision and refinement mode");
    }
    hipStream_t s = H[0]->stream;
    for (int p = 1; p < nh; ++p)
      if (H[p]->stream != s) HIPCHK(hipStreamSynchronize(H[p]->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    const bool fp32 = H[0]->precision == RSS_FP32_REFINE;
    const bool refine = H[0]->refine_steps >= 0;
    std::vector<int> nr(nrhs, nrhs + nh);
    Scratch scr;
    for (auto* h : H) h->stats.last_iters = 0;
    if (!refine) {
      if (!fp32) {
        std::vector<cx<double>*> Z;
        for (int p = 0; p < nh; ++p) Z.push_back((cx<double>*)B[p]);
        apply_batch<double>(H, Z, nr, s);
      } else {
        std::vector<cx<float>*> Z;
        for (int p = 0; p < nh; ++p) {
          const size_t tot = (size_t)H[p]->N * nr[p];
          cx<float>* z = (cx<float>*)scr.alloc(tot * sizeof(cx<float>));
          launch_cast_c64((const cx<double>*)B[p], H[p]->N, nr[p], z, s);
          HIPCHK(hipMemsetAsync(B[p], 0, tot * sizeof(cx<double>), s));
          Z.push_back(z);
        }
        apply_batch<float>(H, Z, nr, s);
        for (int p = 0; p < nh; ++p)
          launch_axpy_from_c64(Z[p], H[p]->N, nr[p], nullptr, (cx<double>*)B[p], s);
      }
      for (auto* h : H) h->stats.last_relres = -1.0;
    } else {
      // x = F^{-1} b, then x += F^{-1} (b - A x) with the FP64 residual, each
      // problem until max_j ||r_j|| / ||b_j|| <= its refine_tol
      std::vector<std::unique_ptr<RefineJob>> jobs;
      for (int p = 0; p < nh; ++p) jobs.emplace_back(refine_begin_impl(H[p], B[p], nr[p], s));
      for (;;) {
        std::vector<RefineJob*> live;
        for (auto& j : jobs)
          if (!j->done) live.push_back(j.get());
        if (live.empty()) break;
        refine_step_impl(live, s);
      }
      for (auto& j : jobs)
        if (refine_finish_impl(j.get(), s) != RSS_OK) code = RSS_ENOCONV;
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    for (auto* h : H) h->stats.t_solve_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
  return rc != RSS_OK ? rc : code;
}

int rss_solve(rss_handle h, void* B, int nrhs) { return rss_solve_batch(1, &h, &B, &nrhs); }

int rss_gridop_create(const rss_kernel* k, int n, double x0, double y0, double h, void* stream,
                      rss_gridop_t* out) {
  if (out) *out = nullptr;
  rss_gridop* op = nullptr;
  const int rc = run([&] {
    if (!out || !k) fail(RSS_EINVAL, "null argument");
    if (n < 1 || n > 2048) fail(RSS_EINVAL, "grid side must be 1 .. 2048");
    if (!(h > 0) || !std::isfinite(h) || !std::isfinite(x0) || !std::isfinite(y0))
      fail(RSS_EINVAL, "bad grid origin or spacing");
    const double pt[2] = {x0 + 0.5 * h, y0 + 0.5 * h};
    validate(pt, 1, k, 1.0, 1);
    if (k->kind == RSS_DEGENERATE) fail(RSS_EUNSUPPORTED, "the grid product needs a translation-invariant kernel");
    op = new rss_gridop();
    op->kern = *k;
    int logm = 1;
    while ((1 << logm) < 2 * n - 1) ++logm;
    GridDesc& g = op->g;
    g.n = n;
    g.M = 1 << logm;
    g.logm = logm;
    g.x0 = x0;
    g.y0 = y0;
    g.h = h;
    g.kp = to_kp(*k);
    if (stream) {
      op->stream = (hipStream_t)stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&op->stream, hipStreamNonBlocking));
      op->own_stream = true;
    }
    const size_t mm = (size_t)g.M * g.M, nn = (size_t)n * n;
    HIPCHK(hipMalloc((void**)&op->ghat, mm * sizeof(cx<double>)));
    HIPCHK(hipMalloc((void**)&op->tw, (size_t)(g.M / 2) * sizeof(cx<double>)));
    HIPCHK(hipMalloc((void**)&op->scale, nn * sizeof(double)));
    HIPCHK(hipMalloc((void**)&op->diag, nn * sizeof(cx<double>)));
    std::vector<cx<double>> tw(g.M / 2);
    for (int i = 0; i < g.M / 2; ++i) {
      const double t = -2.0 * M_PI * (double)i / g.M;
      tw[i] = cx<double>{std::cos(t), std::sin(t)};
    }
    HIPCHK(hipMemcpyAsync(op->tw, tw.data(), tw.size() * sizeof(cx<double>), hipMemcpyHostToDevice, op->stream));
    g.tw = op->tw;
    g.ghat = op->ghat;
    g.scale = op->scale;
    g.diag = op->diag;
    launch_grid_setup(g, op->ghat, op->scale, op->diag, op->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(op->stream));
  });
  if (rc != RSS_OK) {
    delete op;
    return rc;
  }
  *out = op;
  return RSS_OK;
}

int rss_gridop_apply(rss_gridop_t op, const void* X, void* Y, int nrhs) {
  return run([&] {
    if (!op || !X || !Y) fail(RSS_EINVAL, "null argument");
    if (nrhs < 1) fail(RSS_EINVAL, "nrhs must be >= 1");
    op->apply((const cx<double>*)X, nullptr, (cx<double>*)Y, nrhs, 0, op->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(op->stream));
  });
}

int rss_gridop_residual(rss_gridop_t op, const void* X, const void* B, void* R, int nrhs) {
  return run([&] {
    if (!op || !X || !B || !R) fail(RSS_EINVAL, "null argument");
    if (nrhs < 1) fail(RSS_EINVAL, "nrhs must be >= 1");
    op->apply((const cx<double>*)X, (const cx<double>*)B, (cx<double>*)R, nrhs, 1, op->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(op->stream));
  });
}

void rss_gridop_free(rss_gridop_t op) { delete op; }

int rss_set_residual_op(rss_handle h, rss_gridop_t op) {
  return run([&] {
    if (!h) fail(RSS_EINVAL, "null handle");
    if (op && (int64_t)op->g.n * op->g.n != h->N) fail(RSS_EINVAL, "the grid operator has another size");
    h->gridop = op;
  });
}

namespace {
// z = F^{-1} r for one handle (complex128 in and out, r kept), in the handle's precision
void precond_apply(rss_ctx* h, const cx<double>* r, cx<double>* z, int nrhs, cx<float>* zc, hipStream_t s) {
  const size_t tot = (size_t)h->N * nrhs;
  std::vector<rss_ctx*> H{h};
  std::vector<int> nr{nrhs};
  if (h->precision == RSS_FP64) {
    HIPCHK(hipMemcpyAsync(z, r, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
    std::vector<cx<double>*> Z{z};
    apply_batch<double>(H, Z, nr, s);
  } else {
    launch_cast_c64(r, h->N, nrhs, zc, s);
    std::vector<cx<float>*> Z{zc};
    apply_batch<float>(H, Z, nr, s);
    HIPCHK(hipMemsetAsync(z, 0, tot * sizeof(cx<double>), s));
    launch_axpy_from_c64(zc, h->N, nrhs, nullptr, z, s);
  }
}

// per-column conj(x).y, to the host
std::vector<std::complex<double>> coldots(const cx<double>* X, const cx<double>* Y, int64_t N, int nrhs,
                                          cx<double>* part, cx<double>* dout, hipStream_t s) {
  launch_cdot(X, Y, N, nrhs, part, dout, s);
  std::vector<std::complex<double>> v(nrhs);
  HIPCHK(hipMemcpyAsync(v.data(), dout, nrhs * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

cx<double>* up_scalars(const std::vector<std::complex<double>>& v, cx<double>* d, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s));
  return d;
}
}  // namespace

int rss_krylov_ex(rss_handle h, rss_gridop_t A, void* Bv, int nrhs, int method, double tol, int maxit,
                  int restart, void* stream, rss_krylov_stats* st) {
  return run([&] {
    if (!A || !Bv) fail(RSS_EINVAL, "null argument");
    if (nrhs < 1 || maxit < 1 || !(tol > 0) || (method != 0 && method != 1) || restart < 0)
      fail(RSS_EINVAL, "bad Krylov arguments");
    const int64_t N = (int64_t)A->g.n * A->g.n;
    if (h && h->N != N) fail(RSS_EINVAL, "the grid operator has another size");
    const hipStream_t s = h ? h->stream : (stream ? (hipStream_t)stream : A->stream);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    const size_t tot = (size_t)N * nrhs, vb = tot * sizeof(cx<double>);
    cx<double>* B = (cx<double>*)Bv;
    Scratch scr;
    cx<double>* b = (cx<double>*)scr.alloc(vb);
    cx<double>* x = (cx<double>*)scr.alloc(vb);
    cx<double>* z = (cx<double>*)scr.alloc(vb);
    cx<double>* q = (cx<double>*)scr.alloc(vb);
    cx<float>* zc = (h && h->precision != RSS_FP64) ? (cx<float>*)scr.alloc(tot * sizeof(cx<float>)) : nullptr;
    cx<double>* part = (cx<double>*)scr.alloc((size_t)KRYLOV_DOT_BLOCKS * nrhs * sizeof(cx<double>));
    cx<double>* dout = (cx<double>*)scr.alloc((size_t)nrhs * sizeof(cx<double>));
    cx<double>* sa = (cx<double>*)scr.alloc((size_t)nrhs * sizeof(cx<double>));
    cx<double>* sb = (cx<double>*)scr.alloc((size_t)nrhs * sizeof(cx<double>));
    // z = M^{-1} r: the factorization, or the identity without one
    auto precond = [&](const cx<double>* r, cx<double>* out) {
      if (h)
        precond_apply(h, r, out, nrhs, zc, s);
      else
        HIPCHK(hipMemcpyAsync(out, r, vb, hipMemcpyDeviceToDevice, s));
    };
    HIPCHK(hipMemcpyAsync(b, B, vb, hipMemcpyDeviceToDevice, s));
    std::vector<double> bn(nrhs);
    {
      const auto d = coldots(b, b, N, nrhs, part, dout, s);
      for (int c = 0; c < nrhs; ++c) bn[c] = std::sqrt(std::max(0.0, d[c].real()));
    }
    int iters = 0;
    HIPCHK(hipMemsetAsync(x, 0, vb, s));
    if (method == 0) {
      // preconditioned conjugate gradients, the columns in lock step
      cx<double>* r = (cx<double>*)scr.alloc(vb);
      cx<double>* pv = (cx<double>*)scr.alloc(vb);
      HIPCHK(hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, s));
      precond(r, z);
      HIPCHK(hipMemcpyAsync(pv, z, vb, hipMemcpyDeviceToDevice, s));
      std::vector<std::complex<double>> rz = coldots(r, z, N, nrhs, part, dout, s);
      std::vector<char> act(nrhs, 1);
      for (int c = 0; c < nrhs; ++c)
        if (!(bn[c] > 0)) act[c] = 0;
      for (int it = 0; it < maxit; ++it) {
        if (std::find(act.begin(), act.end(), 1) == act.end()) break;
        A->apply(pv, nullptr, q, nrhs, 0, s);
        const auto pq = coldots(pv, q, N, nrhs, part, dout, s);
        std::vector<std::complex<double>> al(nrhs), mal(nrhs);
        for (int c = 0; c < nrhs; ++c) {
          al[c] = act[c] && std::abs(pq[c]) > 0 ? rz[c] / pq[c] : 0.0;
          mal[c] = -al[c];
        }
        launch_caxpby(pv, x, N, nrhs, up_scalars(al, sa, s), nullptr, s);
        launch_caxpby(q, r, N, nrhs, up_scalars(mal, sb, s), nullptr, s);
        iters = it + 1;
        const auto rr = coldots(r, r, N, nrhs, part, dout, s);
        for (int c = 0; c < nrhs; ++c)
          if (act[c] && std::sqrt(std::max(0.0, rr[c].real())) <= tol * bn[c]) act[c] = 0;
        if (std::find(act.begin(), act.end(), 1) == act.end()) break;
        precond(r, z);
        const auto rzn = coldots(r, z, N, nrhs, part, dout, s);
        std::vector<std::complex<double>> be(nrhs);
        for (int c = 0; c < nrhs; ++c) be[c] = act[c] && std::abs(rz[c]) > 0 ? rzn[c] / rz[c] : 0.0;
        launch_caxpby(z, pv, N, nrhs, nullptr, up_scalars(be, sa, s), s);
        rz = rzn;
      }
    } else {
      // right-preconditioned GMRES(m), m = restart (0: no restart), Arnoldi by
      // classical Gram-Schmidt applied twice, the columns in lock step; each
      // cycle starts from the true residual r = b - A x
      const int m = restart > 0 ? std::min(restart, maxit) : maxit;
      const int64_t vstride = (int64_t)tot;
      cx<double>* V = (cx<double>*)scr.alloc((size_t)(m + 1) * vb);
      // with a preconditioner, Z_j = M^{-1} V_j are kept, so that the
      // correction sum_j y_j Z_j needs no further application (the flexible
      // form; the same iterates for a fixed M, one application fewer)
      cx<double>* Zs = h ? (cx<double>*)scr.alloc((size_t)m * vb) : nullptr;
      cx<double>* hcoef = (cx<double>*)scr.alloc((size_t)(m + 1) * nrhs * sizeof(cx<double>));
      using C = std::complex<double>;
      std::vector<char> act(nrhs, 1);
      for (int c = 0; c < nrhs; ++c)
        if (!(bn[c] > 0)) act[c] = 0;
      std::vector<double> rn = bn;  // residual norms at the start of the cycle
      HIPCHK(hipMemcpyAsync(V, b, vb, hipMemcpyDeviceToDevice, s));  // r_0 = b (x_0 = 0)
      while (iters < maxit && std::find(act.begin(), act.end(), 1) != act.end()) {
        const int mc = std::min(m, maxit - iters);
        std::vector<std::vector<C>> H((size_t)nrhs, std::vector<C>((size_t)(mc + 1) * mc, 0.0));
        std::vector<std::vector<C>> cs(nrhs, std::vector<C>(mc)), sn(nrhs, std::vector<C>(mc));
        std::vector<std::vector<C>> gg(nrhs, std::vector<C>(mc + 1, 0.0));
        std::vector<int> kc(nrhs, 0);  // Arnoldi steps of this cycle that count for each column
        std::vector<char> run_c = act;
        auto Hat = [&](int c, int i, int j) -> C& { return H[c][(size_t)j * (mc + 1) + i]; };
        {
          std::vector<C> inv(nrhs);
          for (int c = 0; c < nrhs; ++c) {
            inv[c] = run_c[c] && rn[c] > 0 ? 1.0 / rn[c] : 0.0;
            gg[c][0] = rn[c];
          }
          // V_0 = r / ||r|| (V_0 holds r on entry)
          launch_caxpby(V, V, N, nrhs, up_scalars(inv, sa, s), up_scalars(std::vector<C>(nrhs, 0.0), sb, s), s);
        }
        for (int k = 0; k < mc; ++k) {
          if (std::find(run_c.begin(), run_c.end(), 1) == run_c.end()) break;
          cx<double>* w = V + (size_t)(k + 1) * vstride;
          cx<double>* zk = Zs ? Zs + (size_t)k * vstride : z;
          precond(V + (size_t)k * vstride, zk);
          A->apply(zk, nullptr, w, nrhs, 0, s);
          for (int pass = 0; pass < 2; ++pass) {
            std::vector<C> hv((size_t)(k + 1) * nrhs);
            for (int j = 0; j <= k; ++j) {
              const auto d = coldots(V + (size_t)j * vstride, w, N, nrhs, part, dout, s);
              for (int c = 0; c < nrhs; ++c) {
                hv[(size_t)j * nrhs + c] = d[c];
                Hat(c, j, k) += d[c];
              }
            }
            HIPCHK(hipMemcpyAsync(hcoef, hv.data(), hv.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s));
            launch_lincomb_sub(V, vstride, k + 1, hcoef, w, N, nrhs, s);
          }
          const auto ww = coldots(w, w, N, nrhs, part, dout, s);
          std::vector<C> inv(nrhs);
          for (int c = 0; c < nrhs; ++c) {
            const double hn = std::sqrt(std::max(0.0, ww[c].real()));
            Hat(c, k + 1, k) = hn;
            inv[c] = hn > 0 ? 1.0 / hn : 0.0;
          }
          launch_caxpby(w, w, N, nrhs, up_scalars(inv, sa, s), up_scalars(std::vector<C>(nrhs, 0.0), sb, s), s);
          iters++;
          for (int c = 0; c < nrhs; ++c) {
            if (!run_c[c]) continue;
            // rotations G_i = [[conj(c_i), conj(s_i)], [-s_i, c_i]] (unitary)
            for (int i = 0; i < k; ++i) {
              const C t = std::conj(cs[c][i]) * Hat(c, i, k) + std::conj(sn[c][i]) * Hat(c, i + 1, k);
              Hat(c, i + 1, k) = -sn[c][i] * Hat(c, i, k) + cs[c][i] * Hat(c, i + 1, k);
              Hat(c, i, k) = t;
            }
            const C a = Hat(c, k, k), cc = Hat(c, k + 1, k);
            const double den = std::sqrt(std::norm(a) + std::norm(cc));
            cs[c][k] = den > 0 ? a / den : C(1.0);
            sn[c][k] = den > 0 ? cc / den : C(0.0);
            Hat(c, k, k) = den;
            Hat(c, k + 1, k) = 0.0;
            gg[c][k + 1] = -sn[c][k] * gg[c][k];
            gg[c][k] = std::conj(cs[c][k]) * gg[c][k];
            kc[c] = k + 1;
            if (std::abs(gg[c][k + 1]) <= tol * bn[c] || std::abs(ww[c]) == 0.0) run_c[c] = 0;
          }
        }
        // y = R^{-1} g per column, u = sum_j y_j V_j, x += M^{-1} u
        std::vector<C> ycoef((size_t)(mc + 1) * nrhs, 0.0);
        int kmax = 0;
        for (int c = 0; c < nrhs; ++c) {
          const int mm = kc[c];
          kmax = std::max(kmax, mm);
          std::vector<C> y(mm);
          for (int i = mm - 1; i >= 0; --i) {
            C acc = gg[c][i];
            for (int j = i + 1; j < mm; ++j) acc -= Hat(c, i, j) * y[j];
            y[i] = acc / Hat(c, i, i);
          }
          for (int i = 0; i < mm; ++i) ycoef[(size_t)i * nrhs + c] = -y[i];
        }
        if (kmax > 0) {
          HIPCHK(hipMemcpyAsync(hcoef, ycoef.data(), (size_t)kmax * nrhs * sizeof(cx<double>),
                                hipMemcpyHostToDevice, s));
          if (Zs) {
            // x += sum_j y_j Z_j (hcoef holds -y)
            launch_lincomb_sub(Zs, vstride, kmax, hcoef, x, N, nrhs, s);
          } else {
            HIPCHK(hipMemsetAsync(q, 0, vb, s));
            launch_lincomb_sub(V, vstride, kmax, hcoef, q, N, nrhs, s);
            launch_add_c128(x, q, (int64_t)tot, s);
          }
        }
        // the next cycle's residual, and which columns still iterate
        A->apply(x, b, V, nrhs, 1, s);
        const auto rr = coldots(V, V, N, nrhs, part, dout, s);
        for (int c = 0; c < nrhs; ++c) {
          rn[c] = std::sqrt(std::max(0.0, rr[c].real()));
          if (act[c] && rn[c] <= tol * bn[c]) act[c] = 0;
        }
        if (kmax == 0) break;  // no progress possible (breakdown in every column)
      }
    }
    // the true relative residual of the result
    A->apply(x, b, q, nrhs, 1, s);
    const auto rr = coldots(q, q, N, nrhs, part, dout, s);
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c)
      worst = std::max(worst, bn[c] > 0 ? std::sqrt(std::max(0.0, rr[c].real())) / bn[c] : 0.0);
    HIPCHK(hipMemcpyAsync(B, x, vb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
      st->iters = iters;
      st->relres = worst;
      st->t_ms = ms;
    }
  });
}

int rss_krylov(rss_handle h, rss_gridop_t A, void* Bv, int nrhs, int method, double tol, int maxit,
               rss_krylov_stats* st) {
  if (!h) {
    g_err = "null handle";
    return RSS_EINVAL;
  }
  return rss_krylov_ex(h, A, Bv, nrhs, method, tol, maxit, 0, nullptr, st);
}

void rss_free(rss_handle h) { destroy_ctx(h); }

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
    Scratch scr;
    std::vector<double> hp((size_t)n * 2);
    HIPCHK(hipMemcpyAsync(hp.data(), points, (size_t)n * 2 * sizeof(double), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    const int* tperm = scr.up(spatial_order(hp.data(), n), (hipStream_t)stream);
    residual_batch({{kp, points, n, (const cx<double>*)X, (const cx<double>*)B, (cx<double>*)R, nrhs, tperm}},
                   scr, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  });
}

int rss_residual_static(const rss_kernel* k, const double* points, int64_t n, const void* X,
                        const void* B, void* R, int nrhs, void* stream) {
  return run([&] {
    if (!k || !points || !X || !B || !R) fail(RSS_EINVAL, "null argument");
    if (n < 1 || nrhs < 1) fail(RSS_EINVAL, "bad sizes");
    const hipStream_t st = (hipStream_t)stream;
    char* base = (char*)residual_static_scratch();
    if (!base) fail(RSS_EHIP, "the static scratch of the current device is not available");
    const KParams kp = to_kp(*k);
    // layout of the scratch: target order, descriptor, work items, partial sums
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t tb = (n + 255) / 256;
    auto need = [&](int S) {
      size_t o = up256((size_t)n * sizeof(int)) + up256(sizeof(ResDesc)) +
                 up256((size_t)tb * S * sizeof(ResBlock));
      if (S > 1) o += up256((size_t)tb * sizeof(ResBlock)) + (size_t)S * 16 * n * sizeof(cx<double>);
      return o;
    };
    if (need(1) > RES_STATIC_BYTES)
      fail(RSS_EINVAL, "n = " + std::to_string(n) + " does not fit the static scratch of " +
                           std::to_string(RES_STATIC_BYTES >> 20) + " MiB (about 4 bytes per point)");
    int S = residual_slices(tb);
    while (S > 1 && need(S) > RES_STATIC_BYTES) --S;
    std::vector<double> hp((size_t)n * 2);
    HIPCHK(hipMemcpyAsync(hp.data(), points, (size_t)n * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const std::vector<int> perm = spatial_order(hp.data(), n);
    size_t o = 0;
    int* d_perm = (int*)(base + o);
    o += up256((size_t)n * sizeof(int));
    ResDesc* d_desc = (ResDesc*)(base + o);
    o += up256(sizeof(ResDesc));
    ResBlock* d_blk = (ResBlock*)(base + o);
    o += up256((size_t)tb * S * sizeof(ResBlock));
    ResBlock* d_sum = nullptr;
    cx<double>* d_part = nullptr;
    if (S > 1) {
      d_sum = (ResBlock*)(base + o);
      o += up256((size_t)tb * sizeof(ResBlock));
      d_part = (cx<double>*)(base + o);
    }
    ResDesc e;
    e.kp = kp;
    e.P = points;
    e.n = n;
    e.X = (const cx<double>*)X;
    e.B = (const cx<double>*)B;
    e.R = (cx<double>*)R;
    e.part = d_part;
    e.tperm = d_perm;
    e.nrhs = nrhs;
    e.S = S;
    std::vector<ResBlock> blk, sum;
    for (int64_t t = 0; t < tb; ++t) {
      for (int sp = 0; sp < S; ++sp) blk.push_back({0, (int)t, sp});
      if (S > 1) sum.push_back({0, (int)t, 0});
    }
    HIPCHK(hipMemcpyAsync(d_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_desc, &e, sizeof(ResDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_blk, blk.data(), blk.size() * sizeof(ResBlock), hipMemcpyHostToDevice, st));
    if (S > 1)
      HIPCHK(hipMemcpyAsync(d_sum, sum.data(), sum.size() * sizeof(ResBlock), hipMemcpyHostToDevice, st));
    launch_residual(d_desc, d_blk, (int)blk.size(), d_sum, (int)sum.size(), nrhs, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));  // the host tables above must outlive the copies
  });
}

int rss_set_stream(rss_handle h, void* stream) {
  if (!h || !stream) {
    g_err = "null argument";
    return RSS_EINVAL;
  }
  h->stream = (hipStream_t)stream;
  return RSS_OK;
}

int rss_set_graphs(int enable) { return g_use_graphs.exchange(enable != 0) ? 1 : 0; }

int rss_trim_cache(int64_t* released) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    g_err = "hipGetDevice failed";
    return RSS_EHIP;
  }
  const size_t b = pool().trim(dev);
  if (released) *released = (int64_t)b;
  return RSS_OK;
}

int rss_set_autotune(int enable) {
  if (enable < 0 || enable > 2) {
    g_err = "rss_set_autotune takes 0, 1 or 2";
    return RSS_EINVAL;
  }
  g_autotune.exchange(enable == 1);
  return g_autotune_mode.exchange(enable);
}

int rss_factor_tuning(rss_tune_entry* out, int cap, int* count) {
  if (!count || cap < 0 || (cap > 0 && !out)) {
    g_err = "bad arguments";
    return RSS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_gram_tune_mu);
  int i = 0;
  for (const auto& kv : g_gram_tune) {
    if (i < cap)
      out[i] = {kv.first.prec, kv.first.nb * 16, kv.first.sb, kv.first.rb, kv.second.target, kv.second.chunks,
                kv.second.us};
    ++i;
  }
  *count = i;
  return RSS_OK;
}

int rss_factor_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_gram_tune_mu);
  g_gram_tune.clear();
  return RSS_OK;
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
