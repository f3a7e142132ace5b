// Interpolative decomposition (Def. 1) of a box's compression matrix through
// its Gram matrix, in double-double arithmetic.
//
// The kernels of this library are symmetric, K(x, y) = K(y, x), and so is
// every stored block (A[b2, b] = A[b, b2]^T: the level transition copies or
// evaluates blocks symmetrically, and the Schur updates of eq. e:step keep
// the symmetry because T is real, below).  The compression matrix of
// eqs. e:con / e:proxy, C = [A_{M,B}; A_{B,M}^*; K(proxy, B); K(B, proxy)^*],
// is then [Y; conj(Y)] with Y = [A_{M,B}; K(proxy, B)] (rows permuted), and
//   C^* C = Y^* Y + conj(Y^* Y) = 2 Re(Y^* Y) = 2 Y'^T Y',   Y' = [Re Y; Im Y].
// Column-pivoted QR of C takes its pivots, trailing column norms and
// T = R11^{-1} R12 from C^* C alone (the trailing norms are the diagonal of
// the Schur complements of the Gram matrix, R its pivoted Cholesky factor),
// so the ID of C is the pivoted Cholesky factorization of the real matrix
// G = Y'^T Y' (same pivots, norms scaled by 1/sqrt(2), the same T, which is
// real).  Here
//   * G is accumulated in double-double (every product of two FP32 entries is
//     exact in FP64; FP64 entries use the FMA product error), so the trailing
//     norms near the truncation threshold tol * nu0 keep ~30 digits instead of
//     the ~4 that a plain FP64 Gram matrix keeps at tol = 1e-6;
//   * the Cholesky factorization runs in double-double as well, with the
//     pivot rule of the column-pivoted QR: largest trailing norm, smallest
//     global id within the TIE window, stop when the largest trailing norm is
//     <= tol * nu0 or after min(m, n) steps;
//   * C is never formed: rows of A_{M,B} are read from the stored blocks and
//     the proxy rows evaluated as they are staged.
// Compared with Householder steps on C (a read and a write of the trailing
// m x n matrix per pivot), C is read once and every pivot step works on the
// n x n Gram matrix, held in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "rss_internal.h"

// The error-free transformations below are exact only if every product and
// sum is rounded on its own: no multiply-add contraction anywhere in this
// file (explicit fma() calls are kept).
#pragma clang fp contract(off)

namespace rss {

// ---------------------------------------------------------------------------
// double-double arithmetic (Dekker, Knuth; error-free transformations), with
// explicitly rounded operations so that nothing is contracted into an FMA
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  const double bb = __dsub_rn(s, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(s, bb)), __dsub_rn(b, bb));
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  e = __dsub_rn(b, __dsub_rn(s, a));
}
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = __dmul_rn(a, b);
  e = fma(a, b, -p);
}
// (hi, lo) += p, p an exact product
__device__ __forceinline__ void dd_acc(double& hi, double& lo, double p) {
  double s, e;
  two_sum(hi, p, s, e);
  hi = s;
  lo = __dadd_rn(lo, e);
}
// (hi, lo) += a b for FP64 a, b
__device__ __forceinline__ void dd_acc_prod(double& hi, double& lo, double a, double b) {
  double p, ep, s, e;
  two_prod(a, b, p, ep);
  two_sum(hi, p, s, e);
  hi = s;
  lo = __dadd_rn(lo, __dadd_rn(e, ep));
}
__device__ __forceinline__ void dd_add(double ah, double al, double bh, double bl, double& h, double& l) {
  double s, e;
  two_sum(ah, bh, s, e);
  e = __dadd_rn(e, __dadd_rn(al, bl));
  fast_two_sum(s, e, h, l);
}
__device__ __forceinline__ void dd_mul(double ah, double al, double bh, double bl, double& h, double& l) {
  double p, e;
  two_prod(ah, bh, p, e);
  e = __dadd_rn(e, __dadd_rn(__dmul_rn(ah, bl), __dmul_rn(al, bh)));
  fast_two_sum(p, e, h, l);
}
__device__ __forceinline__ void dd_div(double ah, double al, double bh, double bl, double& h, double& l) {
  const double q1 = ah / bh;
  double ph, pl, rh, rl;
  dd_mul(q1, 0.0, bh, bl, ph, pl);
  dd_add(ah, al, -ph, -pl, rh, rl);
  const double q2 = rh / bh;
  fast_two_sum(q1, q2, h, l);
}
__device__ __forceinline__ void dd_sqrt(double ah, double al, double& h, double& l) {
  if (!(ah > 0.0)) {
    h = l = 0.0;
    return;
  }
  const double q = sqrt(ah);
  double ph, pl, rh, rl;
  two_prod(q, q, ph, pl);
  dd_add(ah, al, -ph, -pl, rh, rl);
  fast_two_sum(q, rh / (2.0 * q), h, l);
}

// ---------------------------------------------------------------------------
// partial Gram matrices: workgroup (slot, chunk, tile group) accumulates
// sum over the chunk's rows y of Y of  Re(y)^T Re(y) + Im(y)^T Im(y)  for NT
// 4 x 4 tiles of the upper triangle.  Rows of Y: the M boxes of B (distance 2,
// ascending offset order, each box's active rows), then the n_proxy proxy
// points w K(y_p, x_j) s_j (s the point scale of the box's columns).  Rows are staged in LDS GRAM_SR at a time, as FP64.
// ---------------------------------------------------------------------------
constexpr int GRAM_SR = 16;

// threads (= 4 x 4 tiles) per workgroup: 192 or 256, whichever launches
// fewer waves for a box's upper triangle (a 64-point box has 136 tiles: one
// workgroup of 3 waves instead of 4, so that four of them share a CU)
int gram_nt(int nmax) {
  const int t = (nmax + 3) / 4, tiles = t * (t + 1) / 2;
  const int w192 = (tiles + 191) / 192 * 3, w256 = (tiles + 255) / 256 * 4;
  return w192 < w256 ? 192 : 256;
}
int gram_tile_groups(int nmax) {
  const int t = (nmax + 3) / 4, nt = gram_nt(std::max(1, nmax));
  return std::max(1, (t * (t + 1) / 2 + nt - 1) / nt);
}

// Three waves per SIMD (at most 168 registers; the spills fall in the row
// staging, not in the accumulation loop): a 64-point box has only 136 tiles,
// so the CU needs more workgroups to keep its SIMDs issuing (Gram time per
// FP32 factorization at 512^2 points with 256-thread workgroups: 21.7 ms at
// two waves per SIMD, 19.9 at three, 20.1 at four; 192-thread workgroups at
// three: 19.2).
template <class R, int NT>
__global__ __launch_bounds__(NT, 3) void k_gram(const Prob<R>* probs, Phase<R> ph, GramWs gw, int ldn) {
  extern __shared__ __align__(16) double gsm[];
  double* sre = gsm;                 // GRAM_SR x ldn
  double* sim = gsm + GRAM_SR * ldn;  // GRAM_SR x ldn
  __shared__ int mbox[16], moff[17], b25[25], n25[25];
  const int slot = blockIdx.x, chunk = blockIdx.y, tg = blockIdx.z;
  const int b = ph.box[slot];
  const Prob<R>& pr = probs[ph.prob[slot]];
  const Level<R> L = pr.L;
  const KParams kp = pr.kp;
  const int n = L.cur[b];
  if (threadIdx.x < 25) {
    const int dx = (int)threadIdx.x % 5 - 2, dy = (int)threadIdx.x / 5 - 2;
    int b2 = -1, cn = 0;
    if (max(abs(dx), abs(dy)) == 2) {
      b2 = box_at(L, b, dx, dy);
      if (b2 >= 0) cn = L.cur[b2];
    }
    b25[threadIdx.x] = b2;
    n25[threadIdx.x] = cn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, o = 0;
    for (int t = 0; t < 25; ++t) {
      if (b25[t] < 0) continue;
      mbox[c] = b25[t];
      moff[c] = o;
      o += n25[t];
      ++c;
    }
    for (int i = c; i < 17; ++i) moff[i] = o;
    for (int i = c; i < 16; ++i) mbox[i] = -1;
  }
  __syncthreads();
  const int sumM = moff[16], npx = pr.n_proxy;
  const int rows = sumM + npx;
  if (chunk == 0 && tg == 0 && threadIdx.x == 0) ph.mrow[slot] = 2 * sumM + 2 * npx;
  if (n == 0) return;
  const bool cplx = kp.kind == 1;  // Laplace and the degenerate kernel are real
  // this thread's 4 x 4 tile (ti <= tj) of the upper triangle
  const int T4 = (n + 3) / 4;
  const int tile = tg * NT + (int)threadIdx.x;
  const bool act = tile < T4 * (T4 + 1) / 2;
  int tj = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while (tj * (tj + 1) / 2 > tile) --tj;
  while ((tj + 1) * (tj + 2) / 2 <= tile) ++tj;
  const int ti = tile - tj * (tj + 1) / 2;
  const int i0 = 4 * ti, j0 = 4 * tj;
  double hi[16], lo[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) hi[e] = lo[e] = 0.0;
  const int r0 = chunk * gw.chunk_rows, r1 = min(rows, r0 + gw.chunk_rows);
  const int* I = L.idx + L.ioff[b];
  const int bx = b % L.nb, by = b / L.nb;
  const double cxx = L.x0 + (bx + 0.5) * L.side, cyy = L.y0 + (by + 0.5) * L.side;
  const double rad = pr.proxy_radius * L.side;
  for (int rb = r0; rb < r1; rb += GRAM_SR) {
    __syncthreads();
    for (int e = threadIdx.x; e < GRAM_SR * n; e += NT) {
      const int rr = e % GRAM_SR, j = e / GRAM_SR, row = rb + rr;
      double re = 0.0, im = 0.0;
      if (row < r1) {
        if (row < sumM) {
          int q = 0;
          while (moff[q + 1] <= row) ++q;
          const int mb = mbox[q];
          const cx<R> v = block_ptr(L, mb, b)[(row - moff[q]) + (int64_t)j * L.n0[mb]];
          re = (double)v.x;
          im = (double)v.y;
        } else {
          const int p = row - sumM;
          const double th = (2.0 * 3.141592653589793116 * p) / npx;
          double sn, cs;
          sincos(th, &sn, &cs);
          const int g = I[j];
          const double px = pr.P[2 * g], py = pr.P[2 * g + 1];
          const cx<double> k = kernel_raw(kp, cxx + rad * cs, cyy + rad * sn, px, py);
          // w K(y_p, x_j) s_j; rounded to the stored precision like the blocks
          const double w = kp.weight * point_scale(kp, px, py);
          const cx<R> v = from_d<R>(w * k.x, w * k.y);
          re = (double)v.x;
          im = (double)v.y;
        }
      }
      sre[rr * ldn + j] = re;
      sim[rr * ldn + j] = im;
    }
    __syncthreads();
    if (!act) continue;
    const int nr = min(GRAM_SR, r1 - rb);
    for (int rr = 0; rr < nr; ++rr) {
      double a[4], c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = sre[rr * ldn + i0 + u];
        c[u] = sre[rr * ldn + j0 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if constexpr (sizeof(R) == sizeof(float)) dd_acc(hi[4 * u + v], lo[4 * u + v], __dmul_rn(a[u], c[v]));
          else dd_acc_prod(hi[4 * u + v], lo[4 * u + v], a[u], c[v]);
        }
      if (cplx) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = sim[rr * ldn + i0 + u];
          c[u] = sim[rr * ldn + j0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if constexpr (sizeof(R) == sizeof(float)) dd_acc(hi[4 * u + v], lo[4 * u + v], __dmul_rn(a[u], c[v]));
            else dd_acc_prod(hi[4 * u + v], lo[4 * u + v], a[u], c[v]);
          }
      }
    }
  }
  if (!act) return;
  double* out = gw.chunks == 1 ? gw.G + gw.oG[slot] : gw.part + gw.oP[slot] + (int64_t)chunk * 2 * n * n;
  const int64_t nn = (int64_t)n * n;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + u, j = j0 + v;
      if (i < n && j < n) {
        out[i + (int64_t)j * n] = hi[4 * u + v];
        out[nn + i + (int64_t)j * n] = lo[4 * u + v];
      }
    }
}

// G = sum of the chunks' partial Gram matrices, in chunk order (deterministic);
// only the upper triangle, the part that k_gram writes and k_chol reads
template <class R>
__global__ __launch_bounds__(256) void k_gram_sum(const Prob<R>* probs, Phase<R> ph, GramWs gw) {
  const int slot = blockIdx.x, b = ph.box[slot];
  const int n = probs[ph.prob[slot]].L.cur[b];
  const int64_t nn = (int64_t)n * n;
  const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (e >= nn || e % n > e / n) return;
  const double* p = gw.part + gw.oP[slot];
  double h = 0.0, l = 0.0;
  for (int c = 0; c < gw.chunks; ++c) dd_add(h, l, p[(int64_t)c * 2 * nn + e], p[(int64_t)c * 2 * nn + nn + e], h, l);
  double* G = gw.G + gw.oG[slot];
  G[e] = h;
  G[nn + e] = l;
}

template <class R>
void launch_gram(const Prob<R>* probs, const Phase<R>& ph, const GramWs& gw, int nmax, hipStream_t s) {
  if (ph.nbox == 0) return;
  const int ldn = ((nmax + 3) / 4) * 4;
  const size_t shm = (size_t)2 * GRAM_SR * ldn * sizeof(double);
  const dim3 grid(ph.nbox, gw.chunks, gram_tile_groups(nmax));
  if (gram_nt(nmax) == 192)
    hipLaunchKernelGGL((k_gram<R, 192>), grid, dim3(192), shm, s, probs, ph, gw, ldn);
  else
    hipLaunchKernelGGL((k_gram<R, 256>), grid, dim3(256), shm, s, probs, ph, gw, ldn);
  if (gw.chunks > 1)
    hipLaunchKernelGGL(k_gram_sum<R>, dim3(ph.nbox, (unsigned)(((int64_t)nmax * nmax + 255) / 256)), dim3(256),
                       0, s, probs, ph, gw);
}

// max / min over the 64 lanes of a wave, in every lane: lane moves within
// rows of 16 lanes (exchange with lane ^ 1, lane ^ 2, then the half-row and
// row mirrors), then shuffles across rows
template <int CTL>
__device__ __forceinline__ int dpp_mov(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTL, 0xF, 0xF, false);
}
template <int CTL>
__device__ __forceinline__ unsigned long long dpp_mov64(unsigned long long x) {
  const int lo = dpp_mov<CTL>((int)(unsigned)x), hi = dpp_mov<CTL>((int)(x >> 32));
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  auto mv = [](T x, auto ctl) {
    unsigned long long u;
    __builtin_memcpy(&u, &x, 8);
    u = dpp_mov64<decltype(ctl)::value>(u);
    T y;
    __builtin_memcpy(&y, &u, 8);
    return y;
  };
  v = op(v, mv(v, std::integral_constant<int, 0xB1>{}));   // lane ^ 1
  v = op(v, mv(v, std::integral_constant<int, 0x4E>{}));   // lane ^ 2
  v = op(v, mv(v, std::integral_constant<int, 0x141>{}));  // 7 - lane in half-rows
  v = op(v, mv(v, std::integral_constant<int, 0x140>{}));  // 15 - lane in rows
  v = op(v, __shfl_xor(v, 16, 64));
  v = op(v, __shfl_xor(v, 32, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ unsigned long long wave_min(unsigned long long v) {
  return wave_reduce(v, [](unsigned long long a, unsigned long long b) { return b < a ? b : a; });
}

// ---------------------------------------------------------------------------
// pivoted Cholesky factorization of G in double-double, one workgroup per box,
// one thread per column, in left-looking form: a pivot step forms only the
// pivot's row of the trailing matrix, from G and the earlier rows of R, and
// updates the trailing diagonal in place.  Per pivot step:
//   * one wave takes the pivot (largest trailing norm sqrt(G_cc) among the
//     remaining columns, smallest global id within TIE of it) and the
//     truncation test against tol * nu0, and forms R(j, p) = sqrt(G(p, p));
//   * the thread of each remaining column c forms
//       G(p, c) - sum_{q < j} R(q, p) R(q, c),  q in increasing order,
//     then R(j, c) = that / R(j, p) and G(c, c) -= R(j, c)^2.
// Each entry takes exactly the double-double operations, in the same order,
// that a right-looking elimination (subtracting R(j, i) R(j, c) from every
// remaining entry after each pivot step) applies to it, so the factorization
// is that one, at O(k^2 n) instead of O(k n^2) work and without writing the
// trailing matrix.  Rows of R (FP64 high and low parts) go to the workspace;
// T = R11^{-1} R12 by back substitution, one thread per redundant column.
// ---------------------------------------------------------------------------
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_chol(const Prob<R>* probs, Phase<R> ph, GramWs gw, int kl) {
  extern __shared__ double2 Rs[];  // rows q < kl of R, (high, low) at q n + c
  __shared__ double dh[GRAM_NMAX], dl[GRAM_NMAX];  // trailing diagonal
  __shared__ double nrm[GRAM_NMAX];                // sqrt(max(dh, 0))
  __shared__ int rem[GRAM_NMAX], piv[GRAM_NMAX], rank[GRAM_NMAX], gidv[GRAM_NMAX];
  __shared__ int sh_p;
  __shared__ double sh_nu0, sh_rh, sh_rl;
  const int slot = blockIdx.x, b = ph.box[slot];
  const Prob<R>& pr = probs[ph.prob[slot]];
  const Level<R> L = pr.L;
  const Records<R> rec = pr.rec;
  const double tol = pr.tol;
  const int n = L.cur[b], m = ph.mrow[slot];
  if (n == 0) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nn = (int64_t)n * n;
  const double* Gg = gw.G + gw.oG[slot];  // upper triangle: G(i, j) at i + j n, i <= j
  double* Rw = gw.Rw + gw.oR[slot];       // row q of R at Rw + q n (high parts)
  double* Rl = Rw + nn;                   // low parts
  const int* gid = L.idx + L.ioff[b];
  const int c = threadIdx.x;  // this thread's column (NT >= n)
  if (c < n) {
    rem[c] = 1;
    gidv[c] = gid[c];
    dh[c] = Gg[c + (int64_t)c * n];
    dl[c] = Gg[nn + c + (int64_t)c * n];
    nrm[c] = sqrt(fmax(dh[c], 0.0));
  }
  __syncthreads();
  int k = 0;
  const int jmax = min(m, n);
  for (int j = 0; j < jmax; ++j) {
    if (wv == 0) {
      double mx = 0.0;
      for (int cc = lane; cc < n; cc += 64)
        if (rem[cc]) mx = fmax(mx, nrm[cc]);
      mx = wave_max(mx);
      if (j == 0 && lane == 0) sh_nu0 = mx;
      const double nu0 = j == 0 ? mx : sh_nu0;
      int best = -1;
      if (!(mx <= tol * nu0)) {
        const double thr = (1.0 - TIE) * mx;
        unsigned long long key = ~0ull;
        for (int cc = lane; cc < n; cc += 64)
          if (rem[cc] && nrm[cc] >= thr) {
            const unsigned long long kc = ((unsigned long long)(unsigned)gidv[cc] << 32) | (unsigned)cc;
            key = kc < key ? kc : key;
          }
        key = wave_min(key);
        best = (int)(unsigned)(key & 0xffffffffu);
      }
      if (lane == 0) {
        sh_p = best;
        if (best >= 0) {
          rem[best] = 0;
          piv[j] = best;
          dd_sqrt(dh[best], dl[best], sh_rh, sh_rl);
        }
      }
    }
    __syncthreads();
    const int p = sh_p;
    if (p < 0) break;
    if (c == p) {
      Rw[(int64_t)j * n + p] = sh_rh;
      if (j < kl) Rs[j * n + p] = double2{sh_rh, sh_rl};  // for the back substitution
    } else if (c < n && rem[c]) {
      const int i0 = min(c, p), i1 = max(c, p);
      double gh = Gg[i0 + (int64_t)i1 * n], gl = Gg[nn + i0 + (int64_t)i1 * n];
      // rows of R in groups of CH, all of a group's loads issued before its
      // subtractions (which stay in row order): rows below kl from LDS, the
      // rest from the workspace.  Past the last row a group subtracts zero,
      // which leaves the double-double (normalized by the subtraction before
      // it) exactly as it is; no branch, so the loads stay ahead of the
      // arithmetic.
      constexpr int CH = 8;
      const int jl = min(j, kl);
      for (int q0 = 0; q0 < jl; q0 += CH) {
        double2 vc[CH], vp[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int q = min(q0 + u, jl - 1);
          vc[u] = Rs[q * n + c];
          vp[u] = Rs[q * n + p];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          double ph_, pl_;
          dd_mul(vc[u].x, vc[u].y, vp[u].x, vp[u].y, ph_, pl_);
          const bool in = q0 + u < jl;
          dd_add(gh, gl, in ? -ph_ : -0.0, in ? -pl_ : -0.0, gh, gl);
        }
      }
      for (int q0 = jl; q0 < j; q0 += CH) {
        double ach[CH], acl[CH], aph[CH], apl[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int64_t o = (int64_t)min(q0 + u, j - 1) * n;
          ach[u] = Rw[o + c];
          acl[u] = Rl[o + c];
          aph[u] = Rw[o + p];
          apl[u] = Rl[o + p];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          double ph_, pl_;
          dd_mul(ach[u], acl[u], aph[u], apl[u], ph_, pl_);
          const bool in = q0 + u < j;
          dd_add(gh, gl, in ? -ph_ : -0.0, in ? -pl_ : -0.0, gh, gl);
        }
      }
      double a, a2;
      dd_div(gh, gl, sh_rh, sh_rl, a, a2);
      Rw[(int64_t)j * n + c] = a;
      Rl[(int64_t)j * n + c] = a2;
      if (j < kl) Rs[j * n + c] = double2{a, a2};
      double ph_, pl_, nh, nl;
      dd_mul(a, a2, a, a2, ph_, pl_);
      dd_add(dh[c], dl[c], -ph_, -pl_, nh, nl);
      dh[c] = nh;
      dl[c] = nl;
      nrm[c] = sqrt(fmax(nh, 0.0));
    }
    __syncthreads();
    k = j + 1;
  }
  __syncthreads();
  const int r = n - k;
  if (threadIdx.x == 0) {
    rec.k[b] = k;
    rec.r[b] = r;
  }
  // ranks by local position (= global id order): skeletons among skeletons,
  // redundant columns among redundant ones
  int* Sloc = ph.Wi + ph.oI[slot];
  const int n0b = L.n0[b];
  int* Rloc = Sloc + n0b;
  for (int a = threadIdx.x; a < n; a += NT) {
    int rk = 0;
    for (int cc = 0; cc < a; ++cc) rk += rem[cc] == rem[a];
    rank[a] = rk;
    if (rem[a]) Rloc[rk] = a;
    else Sloc[rk] = a;
  }
  __syncthreads();
  if (k == 0 || r == 0) return;
  // T = R11^{-1} R12 in place of R12: column c, rows in pivot order; rows of
  // R below kl (high parts) read and overwritten in LDS, the rest in the
  // workspace
  auto rget = [&](int i, int col) { return i < kl ? Rs[i * n + col].x : Rw[(int64_t)i * n + col]; };
  cx<R>* Tout = rec.F + rec.oT[b];
  for (int cc = threadIdx.x; cc < n; cc += NT) {
    if (!rem[cc]) continue;
    for (int i = k - 1; i >= 0; --i) {
      double sacc = rget(i, cc);
      for (int q = i + 1; q < k; ++q) sacc = fma(-rget(i, piv[q]), rget(q, cc), sacc);
      const double x = sacc / rget(i, piv[i]);
      if (i < kl) Rs[i * n + cc].x = x;
      else Rw[(int64_t)i * n + cc] = x;
      Tout[rank[piv[i]] + (int64_t)k * rank[cc]] = from_d<R>(x, 0.0);
    }
  }
}

template <class R>
void launch_chol(const Prob<R>* probs, const Phase<R>& ph, const GramWs& gw, int nmax, hipStream_t s) {
  if (ph.nbox == 0) return;
  static_assert(GRAM_NMAX <= 192, "one thread per column, at most three waves");
  // leading rows of R in LDS: up to 64 KiB per box where many boxes share the
  // CUs, else up to 148 KiB
  const size_t row = (size_t)std::max(1, nmax) * sizeof(double2);
  const size_t budget = ph.nbox >= 256 ? (size_t)64 * 1024 : (size_t)148 * 1024;
  const int kl = (int)std::min<size_t>((size_t)nmax, budget / row);
  const size_t shm = (size_t)kl * row;
  if (nmax <= 64)
    hipLaunchKernelGGL((k_chol<R, 64>), dim3(ph.nbox), dim3(64), shm, s, probs, ph, gw, kl);
  else if (nmax <= 128)
    hipLaunchKernelGGL((k_chol<R, 128>), dim3(ph.nbox), dim3(128), shm, s, probs, ph, gw, kl);
  else
    hipLaunchKernelGGL((k_chol<R, 192>), dim3(ph.nbox), dim3(192), shm, s, probs, ph, gw, kl);
}

template void launch_gram<double>(const Prob<double>*, const Phase<double>&, const GramWs&, int, hipStream_t);
template void launch_gram<float>(const Prob<float>*, const Phase<float>&, const GramWs&, int, hipStream_t);
template void launch_chol<double>(const Prob<double>*, const Phase<double>&, const GramWs&, int, hipStream_t);
template void launch_chol<float>(const Prob<float>*, const Phase<float>&, const GramWs&, int, hipStream_t);

}  // namespace rss
