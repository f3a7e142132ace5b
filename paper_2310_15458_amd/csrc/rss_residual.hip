// The FP64 on-the-fly residual R = B - A X of the refinement (the residual
// whose norm Tab. t:notations reports; refinement stands in for the
// preconditioned iterations of Sec. 5): kernel entries (eq. e:aij) are
// evaluated as they are needed and contracted with X on the matrix cores, so
// A is never stored.  Built in a translation unit of
// its own so that the matrix-core accumulators can be kept in ordinary vector
// registers (see build.py): the near/far branches of the entry evaluation
// inside the source loop otherwise make the compiler copy them between
// register files on every iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "rss_internal.h"

namespace rss {

typedef double mf_d4 __attribute__((ext_vector_type(4)));

// |p - q| for distinct points: the square root of d = dx^2 + dy^2 from the
// hardware reciprocal-square-root estimate, one Goldschmidt step and two
// Newton corrections (the library square root adds range scaling and
// special-case selects that a d of two distinct workload points never needs)
__device__ __forceinline__ double dist_pos(double xi, double yi, double xj, double yj) {
  const double dx = __dsub_rn(xi, xj), dy = __dsub_rn(yi, yj);
  const double d = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
  const double y = __builtin_amdgcn_rsq(d);
  double g = d * y, h = 0.5 * y;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double rr = fma(-g, g, d);
  g = fma(rr, h, g);
  rr = fma(-g, g, d);
  return fma(rr, h, g);
}

// r = b - A x for several problems at once (FP64, entries evaluated on the
// fly), 16 right-hand sides per launch.  Work item = (problem, block of 256
// targets in the order tperm, source slice), split over 256 / RES_TPB
// workgroups; sources stream through LDS RES_SB at a time with their 16
// right-hand-side values.  The contraction runs on the matrix cores: lane l
// evaluates the entry a = ar + i ai for target l mod 16 of a 16-target group
// and source l / 16 of a quad of sources, which is the A operand of
// v_mfma_f64_16x16x4f64 (the B operand: the quad's 16 right-hand-side values
// x = xr + i xi).  The complex product takes three real MFMAs (Gauss's form):
// K1 += (ar + ai) xr, K2 += ar (xi - xr), K3 += ai (xr + xi), and at the end
// a x = (K1 - K3) + i (K1 + K2).  A problem with one slice writes r directly,
// otherwise each slice writes its partial sums and k_residual_sum subtracts
// them from b in slice order.
#ifndef RSS_RES_RG
#define RSS_RES_RG 2
#endif
constexpr int RES_RG = RSS_RES_RG;       // groups of 16 targets per wave
constexpr int RES_TPB = 64 * RES_RG;     // targets per workgroup (a block of 256 spans 256 / RES_TPB)
#ifndef RSS_RES_SB
#define RSS_RES_SB 80
#endif
constexpr int RES_SB = RSS_RES_SB;       // sources per LDS batch
constexpr int RES_TSTRIDE = 2 * (RSS_BESSEL_DEG + 1);  // doubles per interval of the H0 table

// waves per SIMD the register allocation must allow (the LDS footprint of a
// workgroup has to allow as many)
#ifndef RSS_RES_MINW
#define RSS_RES_MINW 4
#endif

__global__ __launch_bounds__(256, RSS_RES_MINW) void k_residual(const ResDesc* dd, const ResBlock* blk, int c0) {
  __shared__ double sx[RES_SB], sy[RES_SB], ssc[RES_SB];
  __shared__ cx<double> xs[RES_SB * 16];
  __shared__ __align__(16) double stab[RSS_BESSEL_NSEG * RES_TSTRIDE];
  const ResBlock bb = blk[blockIdx.x];
  const ResDesc D = dd[bb.prob];
  if (c0 >= D.nrhs) return;
  // the H0 interpolation table, read per lane at data-dependent offsets, staged
  // in LDS; for the Helmholtz kernel scaled so that the two lists give the
  // entry w (i/4) H0 directly: (w/4) J0 (imaginary part) and -(w/4) Y0 or
  // -(w/4) G (real part)
  const KParams kp = D.kp;
  const double w4 = 0.25 * kp.weight;
  for (int e = threadIdx.x; e < RSS_BESSEL_NSEG * RES_TSTRIDE; e += 256)
    stab[e] = kp.kind == 1 ? rss_poly_jy[e] * ((e & 1) ? -w4 : w4) : 0.0;
  const int nc = min(16, D.nrhs - c0);
  const int64_t n = D.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // this lane's target in each of the wave's groups of 16: the A-operand row
  const int64_t base = (int64_t)bb.tb * 256 + (int64_t)blockIdx.y * RES_TPB + wv * 16 * RES_RG;
  double tx[RES_RG], ty[RES_RG], tsc[RES_RG];
  int64_t ti[RES_RG];
#pragma unroll
  for (int g = 0; g < RES_RG; ++g) {
    const int64_t lin = base + g * 16 + li;
    ti[g] = lin < n ? (D.tperm ? (int64_t)D.tperm[lin] : lin) : -1;
    tx[g] = ti[g] >= 0 ? D.P[2 * ti[g]] : 0.0;
    ty[g] = ti[g] >= 0 ? D.P[2 * ti[g] + 1] : 0.0;
    tsc[g] = point_scale(kp, tx[g], ty[g]);  // the point scale s_i of the paper's potential (1 without)
  }
  const int64_t ntile = (n + 255) / 256, per = (ntile + D.S - 1) / D.S;
  const int64_t lo = (int64_t)bb.sp * per * 256, hi = min(n, lo + per * 256);
  mf_d4 k1[RES_RG], k2[RES_RG], k3[RES_RG];
#pragma unroll
  for (int g = 0; g < RES_RG; ++g) {
    k1[g] = mf_d4{0, 0, 0, 0};
    k2[g] = mf_d4{0, 0, 0, 0};
    k3[g] = mf_d4{0, 0, 0, 0};
  }
  for (int64_t t0 = lo; t0 < hi; t0 += RES_SB) {
    __syncthreads();
    if (threadIdx.x < RES_SB) {
      const int64_t sj = t0 + threadIdx.x;
      sx[threadIdx.x] = sj < hi ? D.P[2 * sj] : 0.0;
      sy[threadIdx.x] = sj < hi ? D.P[2 * sj + 1] : 0.0;
      ssc[threadIdx.x] = point_scale(kp, sx[threadIdx.x], sy[threadIdx.x]);
    }
    for (int e = threadIdx.x; e < RES_SB * 16; e += 256) {
      const int sl = e >> 4, c = e & 15;
      const int64_t sj = t0 + sl;
      xs[e] = (sj < hi && c < nc) ? D.X[sj + (int64_t)(c0 + c) * n] : czero<double>();
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)RES_SB, hi - t0);
    for (int q = 0; q < cnt; q += 4) {
      // source q + lk of this quad: the A-operand column and the B-operand row
      const int sl = q + lk;
      const bool sv = sl < cnt;
      const cx<double> xv = xs[sl * 16 + li];
      const double xd1 = xv.y - xv.x, xd2 = xv.x + xv.y;
      const double px = sx[sl], py = sy[sl];
      const int64_t sg = t0 + sl;
#pragma unroll
      for (int g = 0; g < RES_RG; ++g) {
        cx<double> a = czero<double>();
        if (sv && ti[g] >= 0) {
          if (sg == ti[g]) {
            a = diag_entry(kp, tsc[g]);
          } else if (kp.kind == 1) {
            const double x = __dmul_rn(kp.kappa, dist_pos(tx[g], ty[g], px, py));
            if (x < RSS_BESSEL_XA) {
              double pj, pm;  // (w/4) J0 and -(w/4) Y0 (or -(w/4) G)
              const int s = bessel_poly(x, stab, pj, pm);
              if (s < RSS_BESSEL_NLOG) pm = fma(-RSS_TWO_OVER_PI * log(0.5 * x), pj, pm);
              a = cx<double>{pm, pj};
            } else {
              double j0, y0;
              bessel_asym(x, j0, y0);
              a = cx<double>{-w4 * y0, w4 * j0};
            }
          } else {
            const cx<double> kv = kernel_raw(kp, tx[g], ty[g], px, py);
            a = cx<double>{kp.weight * kv.x, kp.weight * kv.y};
          }
          if (kp.bump && sg != ti[g]) {
            const double sc = tsc[g] * ssc[sl];
            a = cx<double>{a.x * sc, a.y * sc};
          }
        }
        k1[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, xv.x, k1[g], 0, 0, 0);
        k2[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, xd1, k2[g], 0, 0, 0);
        k3[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, xd2, k3[g], 0, 0, 0);
      }
    }
  }
  // result row lk + 4 v (target of the group), column li (right-hand side)
#pragma unroll
  for (int g = 0; g < RES_RG; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t lin = base + g * 16 + lk + 4 * v;
      if (lin >= n || li >= nc) continue;
      const int64_t i = D.tperm ? (int64_t)D.tperm[lin] : lin;
      const cx<double> val{k1[g][v] - k3[g][v], k1[g][v] + k2[g][v]};
      if (D.S == 1) {
        const int64_t e = i + (int64_t)(c0 + li) * n;
        D.R[e] = D.B[e] - val;
      } else {
        D.part[((int64_t)bb.sp * 16 + li) * n + i] = val;
      }
    }
}

// r = b - (sum of the slices' partials, in slice order) for the columns
// c0 .. c0 + width - 1; one workgroup per block of 256 targets of a sliced problem
__global__ __launch_bounds__(256) void k_residual_sum(const ResDesc* dd, const ResBlock* blk, int c0,
                                                     int width) {
  const ResBlock bb = blk[blockIdx.x];
  const ResDesc D = dd[bb.prob];
  if (c0 >= D.nrhs) return;
  const int nc = min(width, D.nrhs - c0);  // the columns of this chunk
  const int64_t n = D.n;
  const int64_t i = (int64_t)bb.tb * 256 + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nc; ++c) {
    cx<double> v = D.B[i + (int64_t)(c0 + c) * n];
    for (int sp = 0; sp < D.S; ++sp) v = v - D.part[((int64_t)sp * 16 + c) * n + i];
    D.R[i + (int64_t)(c0 + c) * n] = v;
  }
}

// Scratch of the allocation-free residual (rss_residual_static): its tables,
// target order and partial sums, in one array of every device the library
// runs on (held until the process ends).  Host code reaches it only through
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[RES_STATIC_BYTES];

void* residual_static_scratch() {
  static std::mutex mu;
  static void* ptr[RES_STATIC_MAXDEV] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= RES_STATIC_MAXDEV) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    ptr[dev] = p;
  }
  return ptr[dev];
}

int residual_slices(int64_t target_blocks) {
  if (target_blocks >= 1024) return 1;
  return (int)std::min<int64_t>(16, (1024 + target_blocks - 1) / std::max<int64_t>(target_blocks, 1));
}

void launch_residual(const ResDesc* d, const ResBlock* blk, int nblk, const ResBlock* sum_blk,
                     int nsum, int max_nrhs, hipStream_t s) {
  for (int c0 = 0; c0 < max_nrhs; c0 += 16) {
    hipLaunchKernelGGL(k_residual, dim3(nblk, 256 / RES_TPB), dim3(256), 0, s, d, blk, c0);
    if (nsum > 0)
      hipLaunchKernelGGL(k_residual_sum, dim3(nsum), dim3(256), 0, s, d, sum_blk, c0, std::min(16, max_nrhs - c0));
  }
}

}  // namespace rss
