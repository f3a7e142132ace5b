// Device-side helpers of librss: complex arithmetic, the FP64 kernel-entry
// evaluator (eq. e:aij with the kernels of Sec. 5), and small wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bessel_table.h"

namespace rss {

// ---------------------------------------------------------------------------
// complex numbers over R = double or float
// ---------------------------------------------------------------------------
template <class R>
struct cx {
  R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <class R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
// conj(a) * b
template <class R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// acc += a * b
template <class R>
__device__ __forceinline__ void fma_(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}
// acc += conj(a) * b
template <class R>
__device__ __forceinline__ void fmac_(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.x += a.x * b.x + a.y * b.y;
  acc.y += a.x * b.y - a.y * b.x;
}
template <class R>
__device__ __forceinline__ double abs2d(cx<R> a) {
  return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}
template <class R>
__device__ __forceinline__ cx<R> czero() { return {R(0), R(0)}; }

template <class R>
__device__ __forceinline__ cx<R> from_d(double re, double im) { return {(R)re, (R)im}; }
// widen to / round from complex FP64
template <class R>
__device__ __forceinline__ cx<double> to_d(cx<R> a) { return {(double)a.x, (double)a.y}; }
template <class R>
__device__ __forceinline__ cx<R> from_cd(cx<double> a) { return {(R)a.x, (R)a.y}; }

// ---------------------------------------------------------------------------
// kernel parameters (mirror of the C ABI struct, plain data)
// ---------------------------------------------------------------------------
struct KParams {
  int kind;  // 0 Laplace, 1 Helmholtz, 2 degenerate
  int q;
  double kappa, weight, diag;
  // the paper's discretizations (Sec. 5): point scale s = sqrt(b) of the
  // scattering potential b(x) = exp(-bump_a |x - (bcx, bcy)|^2) when bump != 0,
  // and the diagonal diag + s^2 (cdre + i cdim), (cdre, cdim) = (weight / h^2)
  // times the cell integral of K (0 without cell_diag)
  int bump;
  double bump_a, bcx, bcy;
  double cdre, cdim;
};

// H0^(1)(x) = J0(x) + i Y0(x) for x > 0, in two parts.
// x < XA (bessel_poly): polynomial interpolants (Horner form in t in [-1, 1])
// on intervals of width XA / NSEG, of J0 and of Y0 itself, except on the first
// NLOG intervals, which carry the entire G = Y0 - (2/pi) log(x/2) J0 instead;
// the two coefficient lists come interleaved term by term from `tab`
// (rss_poly_jy, a copy of it in LDS, or such a copy scaled per list).  Returns
// the interval; the caller adds (2/pi) log(x/2) J0 when it is below NLOG.
// x >= XA (bessel_asym): Hankel's large-argument expansion with the phase
// factor e^{i(x - pi/4)} = (cos x + i sin x)(1 - i)/sqrt(2).
constexpr double RSS_TWO_OVER_PI = 0.63661977236758134308;

__device__ __forceinline__ int bessel_poly(double x, const double* tab, double& pj, double& py) {
  constexpr double W = RSS_BESSEL_XA / RSS_BESSEL_NSEG;
  int s = (int)(x * (1.0 / W));
  s = s < RSS_BESSEL_NSEG - 1 ? s : RSS_BESSEL_NSEG - 1;
  // local variable of interval s: (x - (s + 1/2) W) 2 / W, formed as one
  // fused multiply-add 2x/W - (2s + 1) (the same single rounding when W is a
  // power of two)
  const double t = fma(2.0 / W, x, -(double)(2 * s + 1));
  const double* c = tab + s * (2 * (RSS_BESSEL_DEG + 1));
  pj = c[2 * RSS_BESSEL_DEG];
  py = c[2 * RSS_BESSEL_DEG + 1];
#pragma unroll
  for (int k = RSS_BESSEL_DEG - 1; k >= 0; --k) {
    pj = fma(pj, t, c[2 * k]);
    py = fma(py, t, c[2 * k + 1]);
  }
  return s;
}

__device__ __forceinline__ void bessel_asym(double x, double& j0, double& y0) {
  const double ix = 1.0 / x;  // one division; u, Q / x and the amplitude reuse it
  const double u = ix * ix;
  double P = rss_asym_p[RSS_BESSEL_NASYM_HALF - 1];
  double Q = rss_asym_q[RSS_BESSEL_NASYM_HALF - 1];
#pragma unroll
  for (int k = RSS_BESSEL_NASYM_HALF - 2; k >= 0; --k) {
    P = fma(P, u, rss_asym_p[k]);
    Q = fma(Q, u, rss_asym_q[k]);
  }
  Q = Q * ix;
  double sn, cs;
  sincos(x, &sn, &cs);
  constexpr double RS2 = 0.70710678118654752440;
  const double er = (cs + sn) * RS2, ei = (sn - cs) * RS2;
  const double amp = sqrt(RSS_TWO_OVER_PI * ix);
  j0 = amp * (er * P - ei * Q);
  y0 = amp * (er * Q + ei * P);
}

__device__ __forceinline__ void bessel_j0y0(double x, double& j0, double& y0,
                                            const double* tab = rss_poly_jy) {
  if (x < RSS_BESSEL_XA) {
    const int s = bessel_poly(x, tab, j0, y0);
    if (s < RSS_BESSEL_NLOG) y0 = fma(RSS_TWO_OVER_PI * log(0.5 * x), j0, y0);
  } else {
    bessel_asym(x, j0, y0);
  }
}

// Distance with the same rounding as a plain (dx*dx) + (dy*dy): no FMA contraction.
__device__ __forceinline__ double dist_rn(double xi, double yi, double xj, double yj) {
  const double dx = __dsub_rn(xi, xj), dy = __dsub_rn(yi, yj);
  return sqrt(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
}

// K(x_i, x_j) without weight (complex, FP64).
__device__ __forceinline__ cx<double> kernel_raw(const KParams& kp, double xi, double yi, double xj,
                                                 double yj, const double* tab = rss_poly_jy) {
  if (kp.kind == 2) {
    const double dot = __dadd_rn(__dmul_rn(xi, xj), __dmul_rn(yi, yj));
    const double base = 1.0 + dot;
    double p = 1.0;
    for (int e = 0; e < kp.q; ++e) p *= base;
    return {p, 0.0};
  }
  const double r = dist_rn(xi, yi, xj, yj);
  if (kp.kind == 0) {
    constexpr double TWO_PI = 6.283185307179586232;
    return {-log(r) / TWO_PI, 0.0};
  }
  double j0, y0;
  bessel_j0y0(__dmul_rn(kp.kappa, r), j0, y0, tab);
  // (i/4)(J0 + i Y0) = -Y0/4 + i J0/4
  return {-0.25 * y0, 0.25 * j0};
}

// s(x) = sqrt(b(x)) of the scattering potential (1 without one)
__device__ __forceinline__ double point_scale(const KParams& kp, double x, double y) {
  if (!kp.bump) return 1.0;
  const double dx = x - kp.bcx, dy = y - kp.bcy;
  return exp(-0.5 * kp.bump_a * (dx * dx + dy * dy));
}

// A_ii at a point of scale s
__device__ __forceinline__ cx<double> diag_entry(const KParams& kp, double s) {
  const double s2 = s * s;
  return {kp.diag + s2 * kp.cdre, s2 * kp.cdim};
}

// Matrix entry a(i, j) (eq. e:aij): w s_i s_j K off the diagonal (gi != gj),
// the diagonal rule on it.
__device__ __forceinline__ cx<double> entry(const KParams& kp, const double* P, int gi, int gj) {
  if (gi == gj) return diag_entry(kp, point_scale(kp, P[2 * gi], P[2 * gi + 1]));
  cx<double> k = kernel_raw(kp, P[2 * gi], P[2 * gi + 1], P[2 * gj], P[2 * gj + 1]);
  double w = kp.weight;
  if (kp.bump) w *= point_scale(kp, P[2 * gi], P[2 * gi + 1]) * point_scale(kp, P[2 * gj], P[2 * gj + 1]);
  return {w * k.x, w * k.y};
}

// ---------------------------------------------------------------------------
// wave / block reductions (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// slot of the 5x5 stencil for box offset (dx, dy)
__device__ __forceinline__ int slot_of(int dx, int dy) { return (dy + 2) * 5 + (dx + 2); }

}  // namespace rss
