// Device kernels of librss (gfx950).  Every kernel is templated on the real
// type R of the stored matrices (double: complex128 form, float: complex64
// form); kernel entries are always evaluated in FP64 and then rounded.
//
// Per colour phase of one depth the factorization runs
//   build_C -> cpqr -> sparsify -> inverse -> (plan_y, gemm) -> compact -> schur
// over all boxes of the phase at once (one workgroup or more per box).  Boxes
// of one colour are at least three boxes apart, so they read and write
// disjoint blocks (Rem. r:t, Rem. r:nn) and need no synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "rss_internal.h"

namespace rss {

// rows per lane loaded per round in the column loops of the column-pivoted QR
// (one workgroup per box / several workgroups per box)
#ifndef RSS_CPQR_CH
#define RSS_CPQR_CH 8
#endif
#ifndef RSS_CPQR_MG_CH
#define RSS_CPQR_MG_CH 4
#endif
// threads per workgroup of the single- and multi-workgroup QR
#ifndef RSS_CPQR_NT
#define RSS_CPQR_NT 512
#endif
#ifndef RSS_CPQR_MG_NT
#define RSS_CPQR_MG_NT 512
#endif
// columns per wave at a time in the single-workgroup QR (rows per lane per
// round: RSS_CPQR_CH for complex64, half of it for complex128)
#ifndef RSS_CPQR_CB
#define RSS_CPQR_CB 2
#endif
// threads per workgroup of the redundant-block inverse for blocks past 128 rows
#ifndef RSS_INVERSE_NT
#define RSS_INVERSE_NT 512
#endif
// most workgroups per box in the multi-workgroup QR
#ifndef RSS_CPQR_MG_GMAX
#define RSS_CPQR_MG_GMAX 8
#endif
// columns a wave of the multi-workgroup QR updates together
#ifndef RSS_CPQR_MG_CB
#define RSS_CPQR_MG_CB 4
#endif

__device__ __forceinline__ int nb_dx(int j) {  // j-th of the 8 neighbour offsets, ascending id
  const int t = j < 4 ? j : j + 1;
  return t % 3 - 1;
}
__device__ __forceinline__ int nb_dy(int j) {
  const int t = j < 4 ? j : j + 1;
  return t / 3 - 1;
}

// ---------------------------------------------------------------------------
// leaf stencil: A[b, b2] = a(I_b, I_b2) for every pair at distance <= 2
// ---------------------------------------------------------------------------
// One workgroup per (box, problem) for the box's 25 blocks: the polynomial
// table of H0 (15 KiB) is copied to LDS once, and the points of the box and
// of each neighbour in turn (coordinates and scales) are staged there, so an
// entry reads LDS only.  Same arithmetic as entry().  The entries are
// symmetric bit for bit (the distance squares x_i - x_j, which is exactly
// -(x_j - x_i); the point scales multiply in either order), so a box
// evaluates its own block and the blocks toward the 12 neighbours that come
// after it (dy > 0, or dy = 0 and dx > 0) and stores each of those twice,
// A[b, b2] and its transpose A[b2, b].
constexpr int RSS_BESSEL_TAB = RSS_BESSEL_NSEG * 2 * (RSS_BESSEL_DEG + 1);

size_t leaf_assemble_lds(int nmax) { return ((size_t)RSS_BESSEL_TAB + (size_t)6 * nmax) * sizeof(double); }

template <class R>
__global__ __launch_bounds__(256) void k_leaf_assemble(const Prob<R>* probs, int nmax) {
  extern __shared__ double lsm[];
  double* stab = lsm;
  double* pb = stab + RSS_BESSEL_TAB;  // box b: x, y, scale (nmax each)
  double* pc = pb + 3 * nmax;          // the neighbour in turn
  const Level<R> L = probs[blockIdx.y].L;
  const KParams kp = probs[blockIdx.y].kp;
  const double* P = probs[blockIdx.y].P;
  const int b = blockIdx.x;
  if (b >= L.nb * L.nb) return;
  const int m = L.n0[b];
  if (m == 0) return;
  for (int e = threadIdx.x; e < RSS_BESSEL_TAB; e += 256) stab[e] = rss_poly_jy[e];
  {
    const int* I = L.idx + L.ioff[b];
    for (int i = threadIdx.x; i < m; i += 256) {
      const double x = P[2 * I[i]], y = P[2 * I[i] + 1];
      pb[i] = x;
      pb[nmax + i] = y;
      pb[2 * nmax + i] = point_scale(kp, x, y);
    }
  }
  for (int s = 12; s < 25; ++s) {  // the box itself, then the later neighbours
    const int64_t off = L.boff[(int64_t)b * 25 + s];
    if (off < 0) continue;
    const int dx = s % 5 - 2, dy = s / 5 - 2;
    const int b2 = box_at(L, b, dx, dy);
    const int n = L.n0[b2];
    // A[b2, b] (n x m): the slot of offset (-dx, -dy) of box b2
    cx<R>* outT = s == 12 ? nullptr : L.A + L.boff[(int64_t)b2 * 25 + slot_of(-dx, -dy)];
    __syncthreads();  // the previous neighbour's readers are done
    const int* J = L.idx + L.ioff[b2];
    for (int j = threadIdx.x; j < n; j += 256) {
      const double x = P[2 * J[j]], y = P[2 * J[j] + 1];
      pc[j] = x;
      pc[nmax + j] = y;
      pc[2 * nmax + j] = point_scale(kp, x, y);
    }
    __syncthreads();
    cx<R>* out = L.A + off;
    const bool self = s == 12;
    for (int e = threadIdx.x; e < m * n; e += 256) {
      const int i = e % m, j = e / m;
      cx<double> v;
      if (self && i == j) {
        v = diag_entry(kp, pb[2 * nmax + i]);
      } else {
        const cx<double> k = kernel_raw(kp, pb[i], pb[nmax + i], pc[j], pc[nmax + j], stab);
        double w = kp.weight;
        if (kp.bump) w *= pb[2 * nmax + i] * pc[2 * nmax + j];
        v = {w * k.x, w * k.y};
      }
      const cx<R> vr = from_d<R>(v.x, v.y);
      out[i + (int64_t)j * m] = vr;
      if (!self) outT[j + (int64_t)i * n] = vr;
    }
  }
}

// the same with every point read from P (boxes too large for the LDS staging)
template <class R>
__global__ __launch_bounds__(256) void k_leaf_assemble_g(const Prob<R>* probs) {
  const Level<R> L = probs[blockIdx.y].L;
  const KParams kp = probs[blockIdx.y].kp;
  const double* P = probs[blockIdx.y].P;
  const int b = blockIdx.x / 25, s = blockIdx.x % 25;
  if (b >= L.nb * L.nb) return;
  const int64_t off = L.boff[(int64_t)b * 25 + s];
  if (off < 0) return;
  const int b2 = box_at(L, b, s % 5 - 2, s / 5 - 2);
  const int m = L.n0[b], n = L.n0[b2];
  const int* I = L.idx + L.ioff[b];
  const int* J = L.idx + L.ioff[b2];
  cx<R>* out = L.A + off;
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e % m, j = e / m;
    const cx<double> v = entry(kp, P, I[i], J[j]);
    out[i + (int64_t)j * m] = from_d<R>(v.x, v.y);
  }
}

template <class R>
void launch_leaf_assemble(const Prob<R>* probs, int nprob, int max_boxes, int nmax, hipStream_t s) {
  if (nprob == 0) return;
  const size_t shm = leaf_assemble_lds(nmax);
  if (shm <= (size_t)150 * 1024)
    hipLaunchKernelGGL(k_leaf_assemble<R>, dim3(max_boxes, nprob), dim3(256), shm, s, probs, nmax);
  else
    hipLaunchKernelGGL(k_leaf_assemble_g<R>, dim3(max_boxes * 25, nprob), dim3(256), 0, s, probs);
}

// ---------------------------------------------------------------------------
// compression matrix (eqs. e:con, e:proxy):
//   C = [A_{M,B}; A_{B,M}^*; w K(proxy, B) S_B; (w S_B K(B, proxy))^*]
// (S_B the point scales of the box), M boxes in ascending id order, rows of
// each in its active order.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_build_C(const Prob<R>* probs, Phase<R> ph) {
  __shared__ int mbox[16], moff[17];
  __shared__ int b25[25], n25[25];
  const int slot = blockIdx.x, b = ph.box[slot];
  const Prob<R>& pr = probs[ph.prob[slot]];
  const Level<R> L = pr.L;
  const KParams kp = pr.kp;
  const double* P = pr.P;
  const int n = L.cur[b];
  // the boxes of M (distance exactly 2) and their sizes, looked up by 25
  // threads at once; then listed in (dy, dx) order by one thread
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
  const int sumM = moff[16];
  const int npx = pr.n_proxy;
  const int m = 2 * sumM + 2 * npx;
  if (blockIdx.y == 0 && threadIdx.x == 0) ph.mrow[slot] = m;
  const int r0 = blockIdx.y * 64;
  if (r0 >= m || n == 0) return;
  cx<R>* C = ph.W + ph.oC[slot];
  const int* I = L.idx + L.ioff[b];
  const int bx = b % L.nb, by = b / L.nb;
  const double cxx = L.x0 + (bx + 0.5) * L.side, cyy = L.y0 + (by + 0.5) * L.side;
  const double rad = pr.proxy_radius * L.side;
  const int n0b = L.n0[b];
  for (int e = threadIdx.x; e < 64 * n; e += blockDim.x) {
    const int row = r0 + (e & 63), j = e >> 6;
    if (row >= m) continue;
    cx<R> val;
    if (row < 2 * sumM) {
      const int rr = row < sumM ? row : row - sumM;
      int q = 0;
      while (moff[q + 1] <= rr) ++q;
      const int i = rr - moff[q];
      const int mb = mbox[q];
      if (row < sumM) {
        const cx<R>* blk = block_ptr(L, mb, b);  // A[mb, b]: cur[mb] x n, ld n0[mb]
        val = blk[i + (int64_t)j * L.n0[mb]];
      } else {
        const cx<R>* blk = block_ptr(L, b, mb);  // A[b, mb]: n x cur[mb], ld n0[b]
        val = conj(blk[j + (int64_t)i * n0b]);
      }
    } else {
      const int p = (row - 2 * sumM) % npx;
      const bool second = (row - 2 * sumM) >= npx;
      const double th = (2.0 * 3.141592653589793116 * p) / npx;
      double sn, cs;
      sincos(th, &sn, &cs);
      const double gx = cxx + rad * cs, gy = cyy + rad * sn;
      const int g = I[j];
      const double px = P[2 * g], py = P[2 * g + 1];
      const double w = kp.weight * point_scale(kp, px, py);
      if (!second) {
        const cx<double> k = kernel_raw(kp, gx, gy, px, py);
        val = from_d<R>(w * k.x, w * k.y);
      } else {
        const cx<double> k = kernel_raw(kp, px, py, gx, gy);
        val = from_d<R>(w * k.x, -(w * k.y));
      }
    }
    C[row + (int64_t)j * m] = val;
  }
}

template <class R>
void launch_build_C(const Prob<R>* probs, const Phase<R>& ph, int chunks, hipStream_t s) {
  if (ph.nbox == 0) return;
  hipLaunchKernelGGL(k_build_C<R>, dim3(ph.nbox, chunks), dim3(256), 0, s, probs, ph);
}

// ---------------------------------------------------------------------------
// interpolative decomposition by column-pivoted Householder QR (Def. 1):
// exact trailing norms at every step (FP64 accumulation), pivot = smallest
// global id among columns within TIE of the largest norm, stop when the
// largest trailing norm is <= tol * nu0.  Then T = R11^{-1} R12, rows and
// columns reordered to ascending ids.  One workgroup per box.
// ---------------------------------------------------------------------------
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_cpqr(const Prob<R>* probs, Phase<R> ph, int nmax, int vcap) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NW = NT / 64;
  double* nrm = reinterpret_cast<double*>(smem_raw);               // nmax
  double* red = nrm + nmax;                                         // NW
  int* perm = reinterpret_cast<int*>(red + NW);                     // nmax
  int* rankv = perm + nmax;                                         // nmax
  cx<R>* vs = reinterpret_cast<cx<R>*>(smem_raw + (((nmax * 8 + NW * 8 + nmax * 8) + 15) & ~15));
  __shared__ int sh_p;
  __shared__ double sh_nu0;

  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const double tol = probs[ph.prob[slot]].tol;
  const int n = L.cur[b], m = ph.mrow[slot];
  const bool vlds = m <= vcap;
  cx<R>* C = ph.W + ph.oC[slot];
  int* Sloc = ph.Wi + ph.oI[slot];
  const int n0b = L.n0[b];
  int* Rloc = Sloc + n0b;
  const int* gid = L.idx + L.ioff[b];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  for (int c = wv; c < n; c += NW) {
    const cx<R>* col = C + (int64_t)c * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += abs2d(col[i]);
    s = wave_sum(s);
    if (lane == 0) nrm[c] = s;
  }
  for (int c = threadIdx.x; c < n; c += NT) perm[c] = c;
  __syncthreads();
  int k = 0;
  const int jmax = m < n ? m : n;
  for (int j = 0; j < jmax; ++j) {
    if (wv == 0) {
      // largest trailing norm, then the smallest global id within the tie window
      double mx = 0.0;
      for (int c = j + lane; c < n; c += 64) mx = fmax(mx, nrm[c]);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      mx = sqrt(mx);
      if (j == 0 && lane == 0) sh_nu0 = mx;
      const double nu0 = j == 0 ? mx : sh_nu0;
      int best = -1;
      if (!(mx <= tol * nu0)) {
        const double thr = (1.0 - TIE) * mx;
        unsigned long long key = ~0ull;
        for (int c = j + lane; c < n; c += 64)
          if (sqrt(nrm[c]) >= thr) {
            const unsigned long long kc = ((unsigned long long)(unsigned)gid[perm[c]] << 32) | (unsigned)c;
            key = kc < key ? kc : key;
          }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          const unsigned long long ko = __shfl_xor(key, o, 64);
          key = ko < key ? ko : key;
        }
        best = (int)(unsigned)(key & 0xffffffffu);
      }
      if (lane == 0) sh_p = best;
    }
    __syncthreads();
    const int p = sh_p;
    if (p < 0) break;
    if (p != j) {
      cx<R>* cj = C + (int64_t)j * m;
      cx<R>* cp = C + (int64_t)p * m;
      for (int i = threadIdx.x; i < m; i += NT) {
        const cx<R> t = cj[i];
        cj[i] = cp[i];
        cp[i] = t;
      }
      if (threadIdx.x == 0) {
        const int t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
        const double u = nrm[j];
        nrm[j] = nrm[p];
        nrm[p] = u;
      }
    }
    __syncthreads();
    cx<R>* cj = C + (int64_t)j * m;
    double t = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += NT) t += abs2d(cj[i]);
    t = block_sum<NT>(t, red);
    const cx<R> x0 = cj[j];
    const double ax0 = sqrt(abs2d(x0));
    const double xn = sqrt(ax0 * ax0 + t);
    const double phr = ax0 > 0.0 ? (double)x0.x / ax0 : 1.0;
    const double phi = ax0 > 0.0 ? (double)x0.y / ax0 : 0.0;
    const double alr = -phr * xn, ali = -phi * xn;
    const double v0r = (double)x0.x - alr, v0i = (double)x0.y - ali;
    const double vv = v0r * v0r + v0i * v0i + t;
    const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) cj[j] = cx<R>{(R)v0r, (R)v0i};
    __syncthreads();
    const cx<R>* vp = cj + j;
    if (vlds) {
      for (int i = j + threadIdx.x; i < m; i += NT) vs[i - j] = cj[i];
      __syncthreads();
      vp = vs;
    }
    // a wave takes CB columns at a time, CH rows of each per lane per round:
    // CB * CH loads in flight
    constexpr int CH = sizeof(R) == sizeof(double) ? RSS_CPQR_CH / 2 : RSS_CPQR_CH, CB = RSS_CPQR_CB;
    for (int c0 = j + 1 + wv; c0 < n; c0 += NW * CB) {
      cx<R>* col[CB];
      bool on[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        on[u] = c0 + NW * u < n;
        col[u] = C + (int64_t)(on[u] ? c0 + NW * u : c0) * m;
      }
      double dr[CB], di[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) dr[u] = di[u] = 0.0;
      for (int base = j + lane; base < m; base += 64 * CH) {
        cx<R> a[CB][CH];
#pragma unroll
        for (int u = 0; u < CB; ++u)
#pragma unroll
          for (int t = 0; t < CH; ++t)
            if (on[u] && base + 64 * t < m) a[u][t] = col[u][base + 64 * t];
#pragma unroll
        for (int t = 0; t < CH; ++t)
          if (base + 64 * t < m) {
            const cx<R> v = vp[base + 64 * t - j];
#pragma unroll
            for (int u = 0; u < CB; ++u)
              if (on[u]) {
                dr[u] += (double)v.x * a[u][t].x + (double)v.y * a[u][t].y;
                di[u] += (double)v.x * a[u][t].y - (double)v.y * a[u][t].x;
              }
          }
      }
      double sr[CB], si[CB], s2[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        sr[u] = beta * wave_sum(dr[u]);
        si[u] = beta * wave_sum(di[u]);
        s2[u] = 0.0;
      }
      for (int base = j + lane; base < m; base += 64 * CH) {
        cx<R> a[CB][CH];
#pragma unroll
        for (int u = 0; u < CB; ++u)
#pragma unroll
          for (int t = 0; t < CH; ++t)
            if (on[u] && base + 64 * t < m) a[u][t] = col[u][base + 64 * t];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          const int i = base + 64 * t;
          if (i < m) {
            const cx<R> v = vp[i - j];
#pragma unroll
            for (int u = 0; u < CB; ++u)
              if (on[u]) {
                cx<R> x = a[u][t];
                x.x -= (R)((double)v.x * sr[u] - (double)v.y * si[u]);
                x.y -= (R)((double)v.x * si[u] + (double)v.y * sr[u]);
                col[u][i] = x;
                if (i > j) s2[u] += abs2d(x);
              }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const double t2 = wave_sum(s2[u]);
        if (lane == 0 && on[u]) nrm[c0 + NW * u] = t2;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) cj[j] = cx<R>{(R)alr, (R)ali};
    __syncthreads();
    k = j + 1;
  }
  const int r = n - k;
  if (threadIdx.x == 0) {
    rec.k[b] = k;
    rec.r[b] = r;
  }
  // T = R11^{-1} R12 in place of R12, one thread per column
  for (int c = k + threadIdx.x; c < n; c += NT) {
    cx<R>* col = C + (int64_t)c * m;
    for (int i = k - 1; i >= 0; --i) {
      double sr = col[i].x, si = col[i].y;
      for (int l = i + 1; l < k; ++l) {
        const cx<R> a = C[i + (int64_t)l * m], x = col[l];
        sr -= (double)a.x * x.x - (double)a.y * x.y;
        si -= (double)a.x * x.y + (double)a.y * x.x;
      }
      const cx<R> d = C[i + (int64_t)i * m];
      const double dd = (double)d.x * d.x + (double)d.y * d.y;
      col[i] = cx<R>{(R)((sr * d.x + si * d.y) / dd), (R)((si * d.x - sr * d.y) / dd)};
    }
  }
  // ascending local positions of S and R (local order = global id order)
  for (int a = threadIdx.x; a < n; a += NT) {
    const int pa = perm[a];
    const bool isS = a < k;
    const int lo = isS ? 0 : k, hi = isS ? k : n;
    int rk = 0;
    for (int a2 = lo; a2 < hi; ++a2) rk += perm[a2] < pa;
    rankv[a] = rk;
    if (isS) Sloc[rk] = pa;
    else Rloc[rk] = pa;
  }
  __syncthreads();
  if (k > 0 && r > 0) {
    cx<R>* Tout = rec.F + rec.oT[b];
    for (int e = threadIdx.x; e < k * r; e += NT) {
      const int a = e % k, c = e / k;
      Tout[rankv[a] + (int64_t)k * rankv[k + c]] = C[a + (int64_t)(k + c) * m];
    }
  }
}

template <class R>
void launch_cpqr(const Prob<R>* probs, const Phase<R>& ph, int nmax, int mmax, hipStream_t s) {
  if (ph.nbox == 0) return;
  constexpr int NT = RSS_CPQR_NT;
  const size_t head = ((size_t)nmax * 8 + (NT / 64) * 8 + (size_t)nmax * 8 + 15) & ~(size_t)15;
  // the Householder vector is staged in LDS when it fits in 48 KiB
  const int vcap = (int)((48 * 1024) / sizeof(cx<R>));
  const size_t shm = head + (size_t)(mmax < vcap ? mmax : vcap) * sizeof(cx<R>);
  hipLaunchKernelGGL((k_cpqr<R, NT>), dim3(ph.nbox), dim3(NT), shm, s, probs, ph, nmax, vcap);
}

// ---------------------------------------------------------------------------
// The same interpolative decomposition with the rows of each box's C split
// over G workgroups (for depths with few boxes per colour).  Each step the
// workgroups combine partial dot products and partial column norms through
// global memory between two per-box barriers; every workgroup then takes the
// same pivot and truncation decisions from the same sums.  Columns are not
// moved: a permutation (identical in every workgroup) maps positions to
// physical columns.  Barriers spin on a per-box counter with a bounded wait
// (timeout -> error flag, the kernel still exits).  The launch keeps all
// G x boxes workgroups co-resident.
// ---------------------------------------------------------------------------
// bounded wait (the launch's spin limit, ~seconds by default): long enough for
// concurrent work on other streams to drain; a timeout sets the error flag and
// the host redoes the factorization with the single-workgroup QR

// LDS of k_cpqr_mg before the staged Householder vector: three double and two
// int arrays of nmax entries, 16-byte aligned
__host__ __device__ constexpr size_t mg_head_bytes(int nmax) {
  return ((size_t)nmax * (8 * 3 + 8) + 15) & ~(size_t)15;
}
// the staged Householder vector takes up to 48 KiB
template <class R>
constexpr int mg_vcap() { return (int)((48 * 1024) / sizeof(cx<R>)); }

__device__ __forceinline__ void mg_barrier(unsigned* bar, unsigned target, int* err, unsigned spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > spin_limit) {
        atomicOr(err, ERRF_TIMEOUT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

template <class R, int NT>
__global__ __launch_bounds__(NT) void k_cpqr_mg(const Prob<R>* probs, Phase<R> ph, int G, int nmax,
                                                int vcap, double* pnorm, double* pdot,
                                                unsigned* bars, int* err, unsigned spin_limit) {
  constexpr int CH = RSS_CPQR_MG_CH, CB = RSS_CPQR_MG_CB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NW = NT / 64;
  double* nrm = reinterpret_cast<double*>(smem_raw);          // nmax
  double* wre = nrm + nmax;                                     // nmax
  double* wim = wre + nmax;                                     // nmax
  int* perm = reinterpret_cast<int*>(wim + nmax);               // nmax (position -> column)
  int* rankv = perm + nmax;                                     // nmax
  // this workgroup's rows of the current Householder vector (when they fit)
  cx<R>* vsh = reinterpret_cast<cx<R>*>(smem_raw + mg_head_bytes(nmax));
  __shared__ int sh_p;
  __shared__ double sh_nu0;

  const int slot = blockIdx.x / G, g = blockIdx.x % G;
  const int b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const double tol = probs[ph.prob[slot]].tol;
  const int n = L.cur[b], m = ph.mrow[slot];
  cx<R>* C = ph.W + ph.oC[slot];
  int* Sloc = ph.Wi + ph.oI[slot];
  const int n0b = L.n0[b];
  int* Rloc = Sloc + n0b;
  const int* gid = L.idx + L.ioff[b];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rows = (m + G - 1) / G;
  const int r0 = min(m, g * rows), r1 = min(m, r0 + rows);
  double* pn = pnorm + (size_t)slot * G * nmax;   // [g][column]
  double* pd = pdot + (size_t)slot * G * nmax * 2;
  unsigned* bar = bars + slot;
  unsigned nbar = 0;

  for (int c = wv; c < n; c += NW) {
    const cx<R>* col = C + (int64_t)c * m;
    double s = 0.0;
    for (int i = r0 + lane; i < r1; i += 64) s += abs2d(col[i]);
    s = wave_sum(s);
    if (lane == 0) pn[(size_t)g * nmax + c] = s;
  }
  for (int c = threadIdx.x; c < n; c += NT) perm[c] = c;
  mg_barrier(bar, (++nbar) * G, err, spin_limit);
  int k = 0;
  const int jmax = m < n ? m : n;
  for (int j = 0; j < jmax; ++j) {
    for (int c = j + threadIdx.x; c < n; c += NT) {
      const int q = perm[c];
      double s = 0.0;
      for (int h = 0; h < G; ++h) s += pn[(size_t)h * nmax + q];
      nrm[c] = s;
    }
    __syncthreads();
    if (wv == 0) {
      // largest trailing norm, then the smallest global id within the tie window
      double mx = 0.0;
      for (int c = j + lane; c < n; c += 64) mx = fmax(mx, nrm[c]);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      mx = sqrt(mx);
      if (j == 0 && lane == 0) sh_nu0 = mx;
      const double nu0 = j == 0 ? mx : sh_nu0;
      int best = -1;
      if (!(mx <= tol * nu0)) {
        const double thr = (1.0 - TIE) * mx;
        unsigned long long key = ~0ull;
        for (int c = j + lane; c < n; c += 64)
          if (sqrt(nrm[c]) >= thr) {
            const unsigned long long kc = ((unsigned long long)(unsigned)gid[perm[c]] << 32) | (unsigned)c;
            key = kc < key ? kc : key;
          }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          const unsigned long long ko = __shfl_xor(key, o, 64);
          key = ko < key ? ko : key;
        }
        best = (int)(unsigned)(key & 0xffffffffu);
      }
      if (lane == 0) {
        if (best >= 0 && best != j) {
          const int t = perm[j];
          perm[j] = perm[best];
          perm[best] = t;
          const double u = nrm[j];
          nrm[j] = nrm[best];
          nrm[best] = u;
        }
        sh_p = best;
      }
    }
    __syncthreads();
    if (sh_p < 0) break;
    const int pc = perm[j];
    const cx<R>* cj = C + (int64_t)pc * m;
    const cx<R> x0 = cj[j];
    const double ax0 = sqrt(abs2d(x0));
    const double nrm2 = nrm[j];
    const double t = fmax(0.0, nrm2 - ax0 * ax0);
    const double xn = sqrt(nrm2);
    const double phr = ax0 > 0.0 ? (double)x0.x / ax0 : 1.0;
    const double phi = ax0 > 0.0 ? (double)x0.y / ax0 : 0.0;
    const double alr = -phr * xn, ali = -phi * xn;
    const double v0r = (double)x0.x - alr, v0i = (double)x0.y - ali;
    const double vv = v0r * v0r + v0i * v0i + t;
    const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
    const int i0 = max(r0, j);
    // v below the diagonal is the pivot column itself: stage this workgroup's rows
    const bool vl = r1 - i0 <= vcap;
    // row i of v is vsrc[i - i0]: both bases point inside their buffers
    const cx<R>* vsrc = vl ? vsh : cj + i0;
    if (vl) {
      for (int i = i0 + threadIdx.x; i < r1; i += NT) vsh[i - i0] = cj[i];
      __syncthreads();
    }
    // partial dot products v^H C[:, q] over this workgroup's rows: a wave takes
    // CB columns at a time and CH rows of each per lane per round, so that
    // CB * CH loads are in flight
    for (int c0 = j + 1 + wv; c0 < n; c0 += NW * CB) {
      int q[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) q[u] = c0 + NW * u < n ? perm[c0 + NW * u] : -1;
      double dr[CB], di[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) dr[u] = di[u] = 0.0;
      for (int base = i0 + lane; base < r1; base += 64 * CH) {
        cx<R> a[CB][CH];
#pragma unroll
        for (int u = 0; u < CB; ++u)
#pragma unroll
          for (int t = 0; t < CH; ++t)
            if (q[u] >= 0 && base + 64 * t < r1) a[u][t] = C[(int64_t)q[u] * m + base + 64 * t];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          const int i = base + 64 * t;
          if (i < r1) {
            const cx<R> vv = vsrc[i - i0];
            const double vr = (i == j) ? v0r : (double)vv.x;
            const double vi = (i == j) ? v0i : (double)vv.y;
#pragma unroll
            for (int u = 0; u < CB; ++u)
              if (q[u] >= 0) {
                dr[u] += vr * a[u][t].x + vi * a[u][t].y;
                di[u] += vr * a[u][t].y - vi * a[u][t].x;
              }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        dr[u] = wave_sum(dr[u]);
        di[u] = wave_sum(di[u]);
        if (lane == 0 && q[u] >= 0) {
          pd[((size_t)g * nmax + q[u]) * 2] = dr[u];
          pd[((size_t)g * nmax + q[u]) * 2 + 1] = di[u];
        }
      }
    }
    mg_barrier(bar, (++nbar) * G, err, spin_limit);
    for (int c = j + 1 + threadIdx.x; c < n; c += NT) {
      const int q = perm[c];
      double sr = 0.0, si = 0.0;
      for (int h = 0; h < G; ++h) {
        sr += pd[((size_t)h * nmax + q) * 2];
        si += pd[((size_t)h * nmax + q) * 2 + 1];
      }
      wre[c] = beta * sr;
      wim[c] = beta * si;
    }
    __syncthreads();
    // update this workgroup's rows; partial norms of rows > j (columns batched as above)
    for (int c0 = j + 1 + wv; c0 < n; c0 += NW * CB) {
      int q[CB];
      double sr[CB], si[CB], s2[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = c0 + NW * u;
        q[u] = c < n ? perm[c] : -1;
        sr[u] = c < n ? wre[c] : 0.0;
        si[u] = c < n ? wim[c] : 0.0;
        s2[u] = 0.0;
      }
      for (int base = i0 + lane; base < r1; base += 64 * CH) {
        cx<R> a[CB][CH];
#pragma unroll
        for (int u = 0; u < CB; ++u)
#pragma unroll
          for (int t = 0; t < CH; ++t)
            if (q[u] >= 0 && base + 64 * t < r1) a[u][t] = C[(int64_t)q[u] * m + base + 64 * t];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          const int i = base + 64 * t;
          if (i < r1) {
            const cx<R> vv = vsrc[i - i0];
            const double vr = (i == j) ? v0r : (double)vv.x;
            const double vi = (i == j) ? v0i : (double)vv.y;
#pragma unroll
            for (int u = 0; u < CB; ++u)
              if (q[u] >= 0) {
                cx<R> x = a[u][t];
                x.x -= (R)(vr * sr[u] - vi * si[u]);
                x.y -= (R)(vr * si[u] + vi * sr[u]);
                C[(int64_t)q[u] * m + i] = x;
                if (i > j) s2[u] += abs2d(x);
              }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        s2[u] = wave_sum(s2[u]);
        if (lane == 0 && q[u] >= 0) pn[(size_t)g * nmax + q[u]] = s2[u];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && j >= r0 && j < r1) C[j + (int64_t)pc * m] = cx<R>{(R)alr, (R)ali};
    mg_barrier(bar, (++nbar) * G, err, spin_limit);
    k = j + 1;
  }
  // every workgroup leaves the last barrier with the same k and perm; the G
  // workgroups share the columns of T (position c goes to workgroup c mod G)
  const int r = n - k;
  if (g == 0 && threadIdx.x == 0) {
    rec.k[b] = k;
    rec.r[b] = r;
  }
  // T = R11^{-1} R12 (R in rows 0..k-1, columns in pivot order via perm), one
  // thread per column, in place of R12
  cx<R>* Tout = rec.F + rec.oT[b];
  for (int c = k + g + G * (int)threadIdx.x; c < n; c += G * NT) {
    cx<R>* col = C + (int64_t)perm[c] * m;
    for (int i = k - 1; i >= 0; --i) {
      double sr = col[i].x, si = col[i].y;
      for (int l = i + 1; l < k; ++l) {
        const cx<R> a = C[i + (int64_t)perm[l] * m], x = col[l];
        sr -= (double)a.x * x.x - (double)a.y * x.y;
        si -= (double)a.x * x.y + (double)a.y * x.x;
      }
      const cx<R> d = C[i + (int64_t)perm[i] * m];
      const double dd = (double)d.x * d.x + (double)d.y * d.y;
      col[i] = cx<R>{(R)((sr * d.x + si * d.y) / dd), (R)((si * d.x - sr * d.y) / dd)};
    }
  }
  for (int a = threadIdx.x; a < n; a += NT) {
    const int pa = perm[a];
    const bool isS = a < k;
    const int lo = isS ? 0 : k, hi = isS ? k : n;
    int rk = 0;
    for (int a2 = lo; a2 < hi; ++a2) rk += perm[a2] < pa;
    rankv[a] = rk;
    if (g == 0) {
      if (isS) Sloc[rk] = pa;
      else Rloc[rk] = pa;
    }
  }
  __syncthreads();
  // this workgroup's columns of T, copied out in sorted order
  const int rg = r > g ? (r - g + G - 1) / G : 0;
  if (k > 0 && rg > 0) {
    for (int e = threadIdx.x; e < k * rg; e += NT) {
      const int a = e % k, c = g + G * (e / k);
      Tout[rankv[a] + (int64_t)k * rankv[k + c]] = C[a + (int64_t)perm[k + c] * m];
    }
  }
}

__global__ void k_fill_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <class R>
int cpqr_mg_groups(int nbox, int nmax, int mmax) {
  constexpr int NT = RSS_CPQR_MG_NT;
  // one workgroup per compute unit (co-resident when nothing else runs), if
  // this call's LDS allows a workgroup at all
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int per = 0;
  const size_t shm = mg_head_bytes(nmax) + (size_t)mg_vcap<R>() * sizeof(cx<R>);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cpqr_mg<R, NT>, NT, shm);
  const int cap = cus * (per > 0 ? 1 : 0);
  int G = cap / (nbox > 0 ? nbox : 1);
  G = min(G, max(1, mmax / 128));
  // measured at N=512^2: 8 per box beats 4 for phases of up to 16 boxes
  // (15.6 vs 19.3 ms, 13.7 vs 15.6 ms per level), 4 beats 8 for ~28 boxes
  // (20.8 vs 23.5 ms): past 16 boxes the per-step barriers of more groups cost
  // more than their parallel work saves
  return min(G, nbox > 16 ? RSS_CPQR_MG_GMAX / 2 : RSS_CPQR_MG_GMAX);
}

template <class R>
bool launch_cpqr_mg(const Prob<R>* probs, const Phase<R>& ph, int nmax, int mmax, int G,
                    double* pnorm, double* pdot, unsigned* bars, int* err, unsigned spin_limit, hipStream_t s) {
  constexpr int NT = RSS_CPQR_MG_NT;
  if (ph.nbox == 0 || G < 2) return false;
  hipLaunchKernelGGL(k_fill_u32, dim3((ph.nbox + 255) / 256), dim3(256), 0, s, bars, ph.nbox);
  const int vcap = std::min(mg_vcap<R>(), (mmax + G - 1) / G);
  const size_t shm = mg_head_bytes(nmax) + (size_t)vcap * sizeof(cx<R>);
  hipLaunchKernelGGL((k_cpqr_mg<R, NT>), dim3(ph.nbox * G), dim3(NT), shm, s, probs, ph, G, nmax,
                     vcap, pnorm, pdot, bars, err, spin_limit);
  return true;
}

// ---------------------------------------------------------------------------
// sparsification (eq. e:s) with the ID of the box, accumulated in FP64:
//   X_SR = A_SR - A_SS T         X_RS = A_RS - T^* A_SS
//   X_RR = (A_RR - A_RS T) - T^* X_SR
//   X_NR = A_NR - A_NS T         X_RN = A_RN - T^* A_SN
// part 0: the box's own block; part 1 + j: neighbour j (ascending id).
// ---------------------------------------------------------------------------
// sum over s < k of term(s), two accumulators (independent loads in flight)
// out(i, c) = base(i, c) - sum_s G(s, i) t(s, c), i < M, c < r, for the
// products of the sparsification: G(s, i) = g(i, s) (a gathered block of A)
// staged in LDS IC rows i at a time ([s][i], the loads ordered i-fast or
// s-fast as the source is laid out), t = T (k x r, [c][s]) read through tval
// (LDS, or the record when it does not fit; G too is read in place when not
// even two rows fit): a real t, or a complex one, conjugated if CONJ;
// each thread a 2 x 4 tile of outputs, sums in FP64.
template <class R, int NT, bool SFAST, bool GS, bool CONJ, class Tf, class Gf, class Base, class Dst>
__device__ __forceinline__ void sp_gemm(int M, int k, int r, Tf tval, cx<R>* Gs, int IC, Gf g, Base base,
                                        Dst dst) {
  if (!GS) IC = M;  // G read in place (boxes too large to stage two rows)
  for (int i0 = 0; i0 < M; i0 += IC) {
    const int mi = min(IC, M - i0);
    __syncthreads();  // the previous chunk's readers are done
    if (!GS) {
    } else if (SFAST) {
      for (int e = threadIdx.x; e < k * mi; e += NT) {
        const int ss = e % k, i = e / k;
        Gs[ss * IC + i] = g(i0 + i, ss);
      }
    } else {
      for (int e = threadIdx.x; e < k * mi; e += NT) {
        const int i = e % mi, ss = e / mi;
        Gs[ss * IC + i] = g(i0 + i, ss);
      }
    }
    __syncthreads();
    const int np = (mi + 1) / 2, nq = (r + 3) / 4;
    for (int t = threadIdx.x; t < np * nq; t += NT) {
      const int i = 2 * (t % np), c = 4 * (t / np);
      const int i1 = min(i + 1, mi - 1);
      int cc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cc[u] = min(c + u, r - 1) * k;
      cx<double> acc[2][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[0][u] = acc[1][u] = czero<double>();
      for (int ss = 0; ss < k; ++ss) {
        const cx<double> g0 = to_d(GS ? Gs[ss * IC + i] : g(i0 + i, ss));
        const cx<double> g1 = to_d(GS ? Gs[ss * IC + i1] : g(i0 + i1, ss));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const auto tv = tval(cc[u] + ss);
          if constexpr (std::is_same<decltype(tv), const double>::value) {
            acc[0][u].x = fma(g0.x, tv, acc[0][u].x);
            acc[0][u].y = fma(g0.y, tv, acc[0][u].y);
            acc[1][u].x = fma(g1.x, tv, acc[1][u].x);
            acc[1][u].y = fma(g1.y, tv, acc[1][u].y);
          } else if constexpr (CONJ) {  // conj(t) g
            fmac_(acc[0][u], tv, g0);
            fmac_(acc[1][u], tv, g1);
          } else {
            fma_(acc[0][u], g0, tv);
            fma_(acc[1][u], g1, tv);
          }
        }
      }
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i + a2 < mi && c + u < r) dst(i0 + i + a2, c + u, base(i0 + i + a2, c + u) - acc[a2][u]);
    }
  }
}

// Sparsification of box b (eqs. e:con / e:step): with T (k x r) and the
// index lists S, R of the ID,
//   part 0 (the box itself, A = A_bb):
//     X_SR = A_SR - A_SS T           -> rows 0..k-1 of the record's X_{S+N,R}
//     X_RR = A_RR - A_RS T - T^* X_SR (X_SR as stored)
//   part j = 1..8 (neighbour n_j, cn points):
//     X_{n_j R} = A_{n_j R} - A_{n_j S} T, Z_{R n_j} = A_{R n_j} - T^* A_{S n_j}
//   part 9: Z_RS = A_RS - T^* A_SS   -> columns 0..k-1 of Z (r x (k + nN)).
// T is real when the ID came from the Gram matrix (TC false: half the
// arithmetic), complex from the Householder QR (rounding leaves imaginary
// parts there, and the solve uses T as stored, so they are kept).
// Every product runs through sp_gemm; T^* X_SR is formed first (FP64, in the
// phase's FP64 workspace, transposed) and folded into the base of X_RR.
// LDS: the S and R lists, T, then the staging rows.
template <class R, int NT, bool TL, bool GS, bool TC>
__global__ __launch_bounds__(NT) void k_sparsify(const Prob<R>* probs, Phase<R> ph, int nmax, int ic) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int k = rec.k[b], r = rec.r[b];
  if (r == 0) return;
  const int part = blockIdx.y;
  // the 8 neighbours' sizes, loaded together (a missing neighbour reads the
  // box's own entry, then counts 0)
  int nbb[8], ncur[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) nbb[j] = box_at(L, b, nb_dx(j), nb_dy(j));
#pragma unroll
  for (int j = 0; j < 8; ++j) ncur[j] = L.cur[nbb[j] >= 0 ? nbb[j] : b];
  int nN = 0, offj = 0, nbj = -1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (nbb[j] < 0) continue;
    if (j == part - 1) {
      offj = nN;
      nbj = nbb[j];
    }
    nN += ncur[j];
  }
  if (part > 0 && part < 9 && nbj < 0) return;
  const int n0b = L.n0[b];
  using TT = typename std::conditional<TC, cx<double>, double>::type;
  const size_t ib = ((size_t)2 * nmax * sizeof(int) + 15) & ~(size_t)15;
  const size_t tb = TL ? (((size_t)(nmax / 2) * ((nmax + 1) / 2)) * sizeof(TT) + 15) & ~(size_t)15 : 0;
  int* Sl = reinterpret_cast<int*>(smem_raw);
  int* Rl = Sl + k;
  TT* Tl = reinterpret_cast<TT*>(smem_raw + ib);
  cx<R>* Gs = reinterpret_cast<cx<R>*>(smem_raw + ib + tb);
  const cx<R>* Tg = rec.F + rec.oT[b];
  auto tget = [&](int e) -> TT {
    if constexpr (TC) return to_d(Tg[e]);
    else return (double)Tg[e].x;
  };
  {
    const int* Sg = ph.Wi + ph.oI[slot];
    for (int a = threadIdx.x; a < k; a += NT) Sl[a] = Sg[a];
    for (int c = threadIdx.x; c < r; c += NT) Rl[c] = Sg[n0b + c];
    if (TL)
      for (int e = threadIdx.x; e < k * r; e += NT) Tl[e] = tget(e);
  }
  __syncthreads();
  auto tval = [&](int e) -> TT {
    if constexpr (TL) return Tl[e];
    else return tget(e);
  };
  cx<R>* XSNR = rec.F + rec.oXSNR[b];
  const int ldx = k + nN;
  cx<R>* Z = ph.W + ph.oZ[slot];
  const int* gid = L.idx + L.ioff[b];
  if (part == 9) {
    // Z_RS (row a of A_SS read along its columns)
    const cx<R>* A = block_ptr(L, b, b);
    const int ld = n0b;
    sp_gemm<R, NT, true, GS, true>(
        k, k, r, tval, Gs, ic, [&](int a, int s_) { return A[Sl[s_] + (int64_t)Sl[a] * ld]; },
        [&](int a, int c) { return to_d(A[Rl[c] + (int64_t)Sl[a] * ld]); },
        [&](int a, int c, cx<double> v) { Z[c + (int64_t)a * r] = from_cd<R>(v); });
  } else if (part == 0) {
    const cx<R>* A = block_ptr(L, b, b);
    const int ld = n0b;
    // X_SR
    sp_gemm<R, NT, false, GS, false>(
        k, k, r, tval, Gs, ic, [&](int a, int s_) { return A[Sl[a] + (int64_t)Sl[s_] * ld]; },
        [&](int a, int c) { return to_d(A[Sl[a] + (int64_t)Rl[c] * ld]); },
        [&](int a, int c, cx<double> v) { XSNR[a + (int64_t)c * ldx] = from_cd<R>(v); });
    // -(T^* X_SR)^T into the FP64 workspace: W(c2, c1) = -sum_s X_SR(s, c2) conj(T(s, c1))
    cx<double>* Wt = ph.Wd + ph.oD[slot];
    __syncthreads();  // X_SR stored
    sp_gemm<R, NT, true, GS, true>(
        r, k, r, tval, Gs, ic, [&](int c2, int s_) { return XSNR[s_ + (int64_t)c2 * ldx]; },
        [&](int, int) { return czero<double>(); },
        [&](int c2, int c1, cx<double> v) { Wt[c2 + (int64_t)c1 * r] = v; });
    __syncthreads();  // W stored
    // X_RR = A_RR - T^* X_SR - A_RS T
    cx<R>* X = ph.W + ph.oX[slot];
    sp_gemm<R, NT, false, GS, false>(
        r, k, r, tval, Gs, ic, [&](int c1, int s_) { return A[Rl[c1] + (int64_t)Sl[s_] * ld]; },
        [&](int c1, int c2) { return to_d(A[Rl[c1] + (int64_t)Rl[c2] * ld]) + Wt[c2 + (int64_t)c1 * r]; },
        [&](int c1, int c2, cx<double> v) { X[c1 + (int64_t)c2 * r] = from_cd<R>(v); });
    int* gS = rec.G + rec.oS[b];
    int* gR = rec.G + rec.oR[b];
    for (int a = threadIdx.x; a < k; a += NT) gS[a] = gid[Sl[a]];
    for (int c = threadIdx.x; c < r; c += NT) gR[c] = gid[Rl[c]];
    if (threadIdx.x == 0) rec.nN[b] = nN;
  } else {
    const int cn = L.cur[nbj];
    const cx<R>* A1 = block_ptr(L, nbj, b);  // cn x n, ld n0[nbj]
    const int ld1 = L.n0[nbj];
    sp_gemm<R, NT, false, GS, false>(
        cn, k, r, tval, Gs, ic, [&](int i, int s_) { return A1[i + (int64_t)Sl[s_] * ld1]; },
        [&](int i, int c) { return to_d(A1[i + (int64_t)Rl[c] * ld1]); },
        [&](int i, int c, cx<double> v) { XSNR[(k + offj + i) + (int64_t)c * ldx] = from_cd<R>(v); });
    const cx<R>* A2 = block_ptr(L, b, nbj);  // n x cn, ld n0[b]
    sp_gemm<R, NT, true, GS, true>(
        cn, k, r, tval, Gs, ic, [&](int i, int s_) { return A2[Sl[s_] + (int64_t)i * n0b]; },
        [&](int i, int c) { return to_d(A2[Rl[c] + (int64_t)i * n0b]); },
        [&](int i, int c, cx<double> v) { Z[c + (int64_t)(k + offj + i) * r] = from_cd<R>(v); });
    int* gN = rec.G + rec.oN[b];
    const int* gid2 = L.idx + L.ioff[nbj];
    for (int i = threadIdx.x; i < cn; i += NT) gN[offj + i] = gid2[i];
  }
}

template <class R, bool TC>
static void launch_sparsify_t(const Prob<R>* probs, const Phase<R>& ph, int nmax, hipStream_t s) {
  // LDS: the index lists, T (k r <= floor(n/2) ceil(n/2) entries) unless that
  // leaves fewer than 16 staging rows in the cap (then T is read from the
  // record), then as many staging rows (k <= nmax entries each) as the budget
  // leaves: a budget that lets several workgroups share a CU when there are
  // many (the staging loads' latency is hidden by the other workgroups), up
  // to the cap when few.  Boxes too large for two rows read G in place.
  const size_t cap = SPARSIFY_LDS_CAP;
  const size_t ib = sparsify_min_lds(nmax);
  const size_t rowb = (size_t)std::max(1, nmax) * sizeof(cx<R>);
  const size_t te = TC ? sizeof(cx<double>) : sizeof(double);
  size_t tb = (((size_t)(nmax / 2) * ((nmax + 1) / 2)) * te + 15) & ~(size_t)15;
  const bool tl = ib + tb + 16 * rowb <= cap;
  if (!tl) tb = 0;
  const bool gs = ib + 2 * rowb <= cap;
  const int64_t nwg = (int64_t)ph.nbox * 10;
  const dim3 grid(ph.nbox, 10);
  if (!gs) {
    hipLaunchKernelGGL((k_sparsify<R, 256, false, false, TC>), grid, dim3(256), ib, s, probs, ph, nmax, 2);
    return;
  }
  const size_t budget = nwg >= 2048 ? (size_t)32 * 1024 : nwg >= 512 ? (size_t)56 * 1024 : cap;
  const size_t room = budget > ib + tb ? budget - ib - tb : 0;
  const size_t most = cap - ib - tb;  // at least 16 rows with T in LDS, 2 without
  int ic = (int)std::min<size_t>({(size_t)std::max(2, nmax), std::max<size_t>(16, room / rowb), most / rowb});
  ic = std::max(2, ic & ~1);
  const size_t shm = ib + tb + (size_t)ic * rowb;
  // 256 threads per workgroup where there are many, else 1024
  if (nwg >= 512) {
    if (tl) hipLaunchKernelGGL((k_sparsify<R, 256, true, true, TC>), grid, dim3(256), shm, s, probs, ph, nmax, ic);
    else hipLaunchKernelGGL((k_sparsify<R, 256, false, true, TC>), grid, dim3(256), shm, s, probs, ph, nmax, ic);
  } else {
    if (tl) hipLaunchKernelGGL((k_sparsify<R, 1024, true, true, TC>), grid, dim3(1024), shm, s, probs, ph, nmax, ic);
    else hipLaunchKernelGGL((k_sparsify<R, 1024, false, true, TC>), grid, dim3(1024), shm, s, probs, ph, nmax, ic);
  }
}

template <class R>
void launch_sparsify(const Prob<R>* probs, const Phase<R>& ph, int nmax, bool treal, hipStream_t s) {
  if (ph.nbox == 0) return;
  if (treal) launch_sparsify_t<R, false>(probs, ph, nmax, s);
  else launch_sparsify_t<R, true>(probs, ph, nmax, s);
}

// v - c s in complex FP64, four FMAs
__device__ __forceinline__ cx<double> sub_mul(cx<double> v, cx<double> c, cx<double> s) {
  return {fma(-c.x, s.x, fma(c.y, s.y, v.x)), fma(-c.x, s.y, fma(-c.y, s.x, v.y))};
}

// ---------------------------------------------------------------------------
// X_RR^{-1} by Gauss-Jordan elimination with partial pivoting (the LU of
// eq. e:step, kept as an explicit inverse), in FP64 in both forms: X_RR is as
// ill-conditioned as 1 + |T|^2, and an explicit inverse in FP32 costs the
// complex64 form most of its accuracy.  The block is worked on in LDS when it
// fits, else in the phase's FP64 workspace; the result is rounded to the
// record's precision.  One workgroup per box; four barriers per pivot step.
// ---------------------------------------------------------------------------
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_inverse(const Prob<R>* probs, Phase<R> ph, int* errflag,
                                                size_t lds_off, size_t lds_cap, int rmin) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NW = NT / 64;
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  const int slot = blockIdx.x, b = ph.box[slot];
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int r = rec.r[b];
  if (r <= rmin) return;  // empty, or inverted by k_inverse_reg
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // LDS: pivot column, scaled pivot row, pivot rows, column map; then the block if it fits
  cx<double>* colk = reinterpret_cast<cx<double>*>(smem_raw);
  cx<double>* rowk = colk + r;
  int* piv = reinterpret_cast<int*>(rowk + r);
  int* src = piv + r;
  cx<R>* Aout = rec.F + rec.oXi[b];
  const cx<R>* X = ph.W + ph.oX[slot];
  cx<double>* A = (size_t)r * r <= lds_cap ? reinterpret_cast<cx<double>*>(smem_raw + lds_off)
                                          : ph.Wd + ph.oD[slot];
  for (int e = threadIdx.x; e < r * r; e += NT) A[e] = to_d(X[e]);
  const int i0 = threadIdx.x % r, j0 = threadIdx.x / r, di = NT % r, dj = NT / r;
  // wave partials of the pivot search of column kk: for kk = 0 here, later
  // folded into the elimination of step kk - 1
  auto wave_pivot = [&](double best, int bi) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double v2 = __shfl_xor(best, o, 64);
      const int i2 = __shfl_xor(bi, o, 64);
      if (v2 > best || (v2 == best && i2 < bi)) {
        best = v2;
        bi = i2;
      }
    }
    if (lane == 0) {
      rv[wv] = best;
      ri[wv] = bi;
    }
  };
  {
    __syncthreads();
    double best = -1.0;
    int bi = r;
    for (int i = threadIdx.x; i < r; i += NT) {
      const double v = abs2d(A[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    wave_pivot(best, bi);
  }
  __syncthreads();
  for (int kk = 0; kk < r; ++kk) {
    // pivot: largest |A(i, kk)| for i >= kk, smallest i on ties
    double best = rv[0];
    int bi = ri[0];
    bi = ri[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (rv[w] > best || (rv[w] == best && ri[w] < bi)) {
        best = rv[w];
        bi = ri[w];
      }
    if (!(best > 0.0)) {
      if (threadIdx.x == 0) atomicOr(errflag, ERRF_SINGULAR);
      return;  // uniform: every thread reached the same decision
    }
    const int p = bi;
    if (threadIdx.x == 0) piv[kk] = p;
    if (p != kk)
      for (int j = threadIdx.x; j < r; j += NT) {
        const cx<double> t = A[kk + (int64_t)j * r];
        A[kk + (int64_t)j * r] = A[p + (int64_t)j * r];
        A[p + (int64_t)j * r] = t;
      }
    __syncthreads();
    const cx<double> d = A[kk + (int64_t)kk * r];
    const double dd = abs2d(d);
    const cx<double> pinv{d.x / dd, -d.y / dd};
    for (int i = threadIdx.x; i < r; i += NT) {
      colk[i] = A[i + (int64_t)kk * r];
      rowk[i] = i == kk ? pinv : A[kk + (int64_t)i * r] * pinv;
    }
    __syncthreads();
    // every entry once; (i, j) of e = tid + NT t advanced without a division;
    // the entries of column kk + 1 below the diagonal feed the next pivot search
    double nb = -1.0;
    int nbi = r;
    for (int e = threadIdx.x, i = i0, j = j0; e < r * r; e += NT) {
      cx<double> v;
      if (i == kk) v = rowk[j];
      else if (j == kk) v = czero<double>() - colk[i] * pinv;
      else v = sub_mul(A[e], colk[i], rowk[j]);
      A[e] = v;
      if (j == kk + 1 && i > kk) {
        const double a2 = abs2d(v);
        if (a2 > nb || (a2 == nb && i < nbi)) {
          nb = a2;
          nbi = i;
        }
      }
      i += di;
      j += dj;
      if (i >= r) {
        i -= r;
        ++j;
      }
    }
    wave_pivot(nb, nbi);
    __syncthreads();
  }
  // undo the row interchanges as column interchanges in reverse order: final
  // column c is column src[c] of the eliminated block
  if (threadIdx.x == 0) {
    for (int c = 0; c < r; ++c) src[c] = c;
    for (int kk = r - 1; kk >= 0; --kk) {
      const int p = piv[kk], t = src[kk];
      src[kk] = src[p];
      src[p] = t;
    }
  }
  __syncthreads();
  for (int c = wv; c < r; c += NW) {
    const cx<double>* Ac = A + (int64_t)src[c] * r;
    for (int i = lane; i < r; i += 64) Aout[i + (int64_t)c * r] = from_cd<R>(Ac[i]);
  }
}

// lane moves within rows of 16 lanes (DPP controls): exchange with lane ^ 1,
// with lane ^ 2, lane i with 7 - i of its half-row, lane i with 15 - i
enum { DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141 };
template <int CTL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTL, 0xF, 0xF, false);
}
template <int CTL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = dpp_i<CTL>((int)(unsigned)u), hi = dpp_i<CTL>((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// The same elimination for blocks held in registers: a TI x TJ grid of
// threads, thread (ti, tj) owning the entries (ti + TI a, tj + TJ c),
// a < RA, c < RC, for blocks of up to min(TI RA, TJ RC) rows.  Rows are not
// interchanged: the pivot row of step kk stays where it is and two tables
// (the position of each row in the row-interchanging form above, and the row
// at each position) record the interchanges, so the pivot choices and their
// tie rule are those of k_inverse.  Entry (i, j) of the eliminated block is
// entry (position of i, row at position j) of the inverse.
// A step has two barriers: after the pivot row (scaled) is posted to LDS, and
// after the next pivot is chosen.  The TI threads holding column kk + 1 (a
// wave's lanes) update that column first, post it for the next step and
// choose its pivot with its reciprocal while the other waves update the
// rest; every entry is updated as v - c s, and the pivot row and column are
// then rewritten by the few threads holding them.  The steps are unrolled by
// column block, so that the blocks of columns kk and kk + 1 are known at
// compile time.
template <class R, int TI, int TJ, int RA, int RC>
__global__ __launch_bounds__(TI * TJ) void k_inverse_reg(const Prob<R>* probs, Phase<R> ph, int* errflag) {
  static_assert(TI == 16 || TI == 32, "a column's holders are one or two rows of lanes of a wave");
  constexpr int RM = TI * RA < TJ * RC ? TI * RA : TJ * RC;
  constexpr int NT = TI * TJ;
  __shared__ cx<double> colk[2][TI * RA], rowk[TJ * RC];
  __shared__ int pos[TI * RA], rowat[TI * RA];
  __shared__ double selv[2];
  __shared__ int selr[2];
  __shared__ cx<double> selinv[2];  // 1 / the chosen pivot
  const int slot = blockIdx.x, b = ph.box[slot];
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int r = rec.r[b];
  if (r == 0 || r > RM) return;  // larger blocks: k_inverse
  const int ti = (int)threadIdx.x % TI, tj = (int)threadIdx.x / TI;
  const cx<R>* X = ph.W + ph.oX[slot];
  cx<double> v[RA][RC];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      const int i = ti + TI * a, j = tj + TJ * c;
      v[a][c] = (i < r && j < r) ? to_d(X[i + (int64_t)j * r]) : czero<double>();
    }
  for (int i = threadIdx.x; i < TI * RA; i += NT) {
    pos[i] = i;
    rowat[i] = i;
  }
  // by the TI threads holding column c (block C of their entries): post the
  // column to colk[c & 1] and choose its pivot among the rows at positions
  // >= c (largest |.|^2, the smallest position on ties) into slot c & 1 with
  // its reciprocal, then interchange positions c and that of the pivot row.
  // The choice is a reduction over the TI lanes: lane moves within rows of
  // 16 lanes (quad exchanges, then the half-row and row mirrors), and a
  // shuffle between the two rows of a 32-lane group.
  auto post_and_search = [&](auto Cc, int c) __attribute__((always_inline)) {
    constexpr int C = decltype(Cc)::value;
    const int q = rowat[c];
    double best = -1.0, dx = 0.0, dy = 0.0;
    int key = 0;  // position * 256 + row
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = ti + TI * a;
      colk[c & 1][i] = v[a][C];
      if (i >= r) continue;
      const int pi = pos[i];
      const double a2 = abs2d(v[a][C]);
      const int k2 = pi * 256 + i;
      if (pi >= c && (a2 > best || (a2 == best && k2 < key))) {
        best = a2;
        key = k2;
        dx = v[a][C].x;
        dy = v[a][C].y;
      }
    }
    auto take = [&](double b2, int k2, double x2, double y2) __attribute__((always_inline)) {
      if (b2 > best || (b2 == best && k2 < key)) {
        best = b2;
        key = k2;
        dx = x2;
        dy = y2;
      }
    };
    auto dpp_round = [&](auto Ctl) __attribute__((always_inline)) {
      constexpr int CTL = decltype(Ctl)::value;
      take(dpp_d<CTL>(best), dpp_i<CTL>(key), dpp_d<CTL>(dx), dpp_d<CTL>(dy));
    };
    dpp_round(std::integral_constant<int, DPP_QUAD_XOR1>{});
    dpp_round(std::integral_constant<int, DPP_QUAD_XOR2>{});
    dpp_round(std::integral_constant<int, DPP_ROW_HALF_MIRROR>{});
    dpp_round(std::integral_constant<int, DPP_ROW_MIRROR>{});
    if constexpr (TI == 32)
      take(__shfl_xor(best, 16, 64), __shfl_xor(key, 16, 64), __shfl_xor(dx, 16, 64), __shfl_xor(dy, 16, 64));
    if (ti == 0) {
      const int pr = key & 255, pp = key >> 8;
      const double inv = 1.0 / best;
      selv[c & 1] = best;
      selr[c & 1] = pr;
      selinv[c & 1] = cx<double>{dx * inv, -dy * inv};
      if (best > 0.0) {
        rowat[c] = pr;
        rowat[pp] = q;
        pos[pr] = c;
        pos[q] = pp;
      }
    }
  };
  // step kk, its column in block KB and column kk + 1 in block C1; false if
  // the block is singular
  auto step = [&](auto KBc, auto C1c, int kk) __attribute__((always_inline)) -> bool {
    constexpr int KB = decltype(KBc)::value, C1 = decltype(C1c)::value;
    const int buf = kk & 1;
    __syncthreads();
    const double best = selv[buf];
    const int p = selr[buf];
    if (!(best > 0.0)) return false;  // uniform: every thread read the same pivot
    const cx<double> pinv = selinv[buf];
    const bool prow = ti == p % TI, pcol = tj == kk % TJ;
    const int ap = p / TI;
    // The row of v at the runtime block ap is reached by one branch per
    // block; the empty asm with the block number keeps the compiler from
    // merging the branches into an access through a selected pointer, which
    // would move v out of registers.
    if (prow) {  // the pivot row, scaled: row p of the result
      static_for<0, RA>([&](auto Ac) __attribute__((always_inline)) {
        constexpr int A = decltype(Ac)::value;
        if (A == ap) {
#pragma unroll
          for (int c = 0; c < RC; ++c) rowk[tj + TJ * c] = (c == KB && pcol) ? pinv : v[A][c] * pinv;
          __asm__ volatile("; row block %0" ::"i"(A));
        }
      });
    }
    __syncthreads();
    cx<double> rs[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) rs[c] = rowk[tj + TJ * c];
    const cx<double>* col = colk[buf] + ti;  // column kk at rows ti + TI a
    // column kk + 1 first, by its holders (its final values: row p included)
    const bool first = kk + 1 < r && tj == (kk + 1) % TJ;
    if (first) {
#pragma unroll
      for (int a = 0; a < RA; ++a)
        v[a][C1] = ti + TI * a == p ? rs[C1] : sub_mul(v[a][C1], col[TI * a], rs[C1]);
      post_and_search(C1c, kk + 1);
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const cx<double> ca = col[TI * a];
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c != C1) v[a][c] = sub_mul(v[a][c], ca, rs[c]);
      if (!first) v[a][C1] = sub_mul(v[a][C1], ca, rs[C1]);
    }
    if (pcol) {
#pragma unroll
      for (int a = 0; a < RA; ++a) v[a][KB] = czero<double>() - col[TI * a] * pinv;
    }
    if (prow) {
      static_for<0, RA>([&](auto Ac) __attribute__((always_inline)) {
        constexpr int A = decltype(Ac)::value;
        if (A == ap) {
#pragma unroll
          for (int c = 0; c < RC; ++c) v[A][c] = rs[c];
          __asm__ volatile("; row block %0" ::"i"(A));
        }
      });
    }
    return true;
  };
  __syncthreads();
  if (tj == 0) post_and_search(std::integral_constant<int, 0>{}, 0);
  bool ok = true;
  static_for<0, RC>([&](auto KBc) __attribute__((always_inline)) {
    constexpr int KB = decltype(KBc)::value;
    constexpr int NB = KB + 1 < RC ? KB + 1 : KB;  // block of the column after this block
    for (int kr = 0; ok && kr < TJ - 1 && KB * TJ + kr < r; ++kr) ok = step(KBc, KBc, KB * TJ + kr);
    if (ok && KB * TJ + TJ - 1 < r) ok = step(KBc, std::integral_constant<int, NB>{}, KB * TJ + TJ - 1);
  });
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(errflag, ERRF_SINGULAR);
    return;
  }
  __syncthreads();
  cx<R>* Aout = rec.F + rec.oXi[b];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      const int i = ti + TI * a, j = tj + TJ * c;
      if (i < r && j < r) Aout[pos[i] + (int64_t)rowat[j] * r] = from_cd<R>(v[a][c]);
    }
}

template <class R>
void launch_inverse(const Prob<R>* probs, const Phase<R>& ph, int* errflag, int nmax,
                    hipStream_t s) {
  if (ph.nbox == 0) return;
  // blocks of up to 128 rows in registers: 1024 threads (2 x 2, 3 x 3 or
  // 4 x 4 entries each), 512 (2 x 4) where many boxes share the CUs
  int rreg;
  if (nmax <= 64 && ph.nbox >= 256) {
    hipLaunchKernelGGL((k_inverse_reg<R, 32, 16, 2, 4>), dim3(ph.nbox), dim3(512), 0, s, probs, ph, errflag);
    rreg = 64;
  } else if (nmax <= 64) {
    hipLaunchKernelGGL((k_inverse_reg<R, 32, 32, 2, 2>), dim3(ph.nbox), dim3(1024), 0, s, probs, ph, errflag);
    rreg = 64;
  } else if (nmax <= 96) {
    hipLaunchKernelGGL((k_inverse_reg<R, 32, 32, 3, 3>), dim3(ph.nbox), dim3(1024), 0, s, probs, ph, errflag);
    rreg = 96;
  } else {
    hipLaunchKernelGGL((k_inverse_reg<R, 32, 32, 4, 4>), dim3(ph.nbox), dim3(1024), 0, s, probs, ph, errflag);
    rreg = 128;
  }
  if (nmax <= rreg) return;
  const size_t E = sizeof(cx<double>);
  const size_t head = ((size_t)nmax * (2 * E + 2 * sizeof(int)) + 15) & ~(size_t)15;
  // the block itself in LDS up to 96 KiB (r <= 78) where many boxes share the
  // CUs; with few boxes (one workgroup per CU anyway) up to the LDS size
  const size_t lim = ph.nbox <= 512 ? (size_t)(158 * 1024) : (size_t)(150 * 1024);
  const size_t room = head < lim ? lim - head : 0;
  const size_t cap = std::min({(size_t)nmax * nmax, ph.nbox <= 512 ? room / E : (size_t)(96 * 1024) / E, room / E});
  const size_t shm = head + cap * E;
  hipLaunchKernelGGL((k_inverse<R, RSS_INVERSE_NT>), dim3(ph.nbox), dim3(RSS_INVERSE_NT), shm, s, probs, ph,
                     errflag, head, cap, rreg);
}

// ---------------------------------------------------------------------------
// GEMM descriptors
// ---------------------------------------------------------------------------
template <class R>
__global__ void k_plan_y(const Prob<R>* probs, Phase<R> ph, GemmDesc<R>* desc) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= ph.nbox) return;
  const int b = ph.box[slot];
  const Records<R>& rec = probs[ph.prob[slot]].rec;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  GemmDesc<R> d;
  d.C = rec.F + rec.oY[b];
  d.A = rec.F + rec.oXi[b];
  d.B = ph.W + ph.oZ[slot];
  d.ldc = r > 0 ? r : 1;
  d.lda = d.ldc;
  d.ldb = d.ldc;
  d.M = r;
  d.N = r > 0 ? k + nN : 0;
  d.K = r;
  d.beta = 0;
  d.sign = 1;
  desc[slot] = d;
}

template <class R>
void launch_plan_y(const Prob<R>* probs, const Phase<R>& ph, GemmDesc<R>* desc, hipStream_t s) {
  if (ph.nbox == 0) return;
  hipLaunchKernelGGL(k_plan_y<R>, dim3((ph.nbox + 63) / 64), dim3(64), 0, s, probs, ph, desc);
}

// Schur complement update (eq. e:step, Rem. r:nn):
//   block(t1, t2) -= [X_SR; X_NR](rows of t1) * Y(:, cols of t2)
// for t1, t2 in {B} u N(B); B's own rows/columns are its skeletons.

// ---------------------------------------------------------------------------
// batched ragged complex GEMM on the matrix cores: C = (beta C) + sign * A B.
// 64 x 64 tiles, 16-deep K slices staged in LDS; each of the 4 waves owns a
// 32 x 32 quarter as 2 x 2 blocks of 16 x 16 and computes the transposed
// block B^T A^T with the 16x16x4 MFMA (so that consecutive lanes hold
// consecutive rows of the column-major C).  Complex products take four real
// MFMAs: re += br ar - bi ai, im += bi ar + br ai.  In the complex64 form each
// K slice is accumulated in FP32 and the slices are added in FP64.
// ---------------------------------------------------------------------------
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <class R>
struct Mfma;
template <>
struct Mfma<double> {
  typedef mf_d4 acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in slot v of lane l
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef mf_f4 acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// write sink of the read-modify-write epilogue below: one complex128 slot per
// thread of a 256-thread workgroup, never read for a result
__device__ __align__(16) double rss_rmw_sink[2 * 256];

// One 64 x 64 tile of C(i0 + ., j0 + .) = A (M x K, leading dimension lda)
// times B (K x N, ldb): four waves, each a 32 x 32 quarter on the matrix cores
// (4 real MFMAs per complex product), K in slices of 16 staged in LDS, the
// next slice's loads in flight during the current slice's MFMAs, and no MFMA
// steps past K in the last slice.  The waves compute B^T A^T so that
// consecutive lanes hold consecutive rows of C; emit(i, j, re, im) receives
// every element inside M x N (complex64 form: the K slices summed in FP64).
// With sub_at given instead (a functor (i, j) -> cx<R>*), each element times
// sub_scale is subtracted from *sub_at(i, j): all of a lane's 16 targets are
// loaded before any is stored, so the read-modify-writes overlap instead of
// taking one memory round trip each.
template <class R, class Emit, class SubAt = std::nullptr_t>
__device__ __forceinline__ void gemm_tile(const cx<R>* A, int lda, const cx<R>* B, int ldb, int Mr, int Nc, int K,
                                          int i0, int j0, Emit&& emit, SubAt sub_at = nullptr,
                                          double sub_scale = 1.0) {
  using M = Mfma<R>;
  using acc_t = typename M::acc;
  __shared__ cx<R> As[16][64];
  __shared__ cx<R> Bs[16][65];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  acc_t cr[2][2], ci[2][2];
  double fr[2][2][4], fi[2][2][4];  // complex64 form: FP64 sum of the slices
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = acc_t{0, 0, 0, 0};
      ci[a][b] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) fr[a][b][v] = fi[a][b][v] = 0.0;
    }
  // this thread's four A and four B entries of a K slice, loaded into
  // registers one slice ahead so that the loads overlap the previous slice's
  // MFMAs
  cx<R> ra[4], rb[4];
  auto load_slice = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int i = e & 63, kk = e >> 6;
      const int gi = i0 + i, gk = k0 + kk;
      ra[u] = (gi < Mr && gk < K) ? A[gi + (int64_t)gk * lda] : czero<R>();
      const int kb = e & 15, j = e >> 4;
      const int gj = j0 + j, gkb = k0 + kb;
      rb[u] = (gj < Nc && gkb < K) ? B[gkb + (int64_t)gj * ldb] : czero<R>();
    }
  };
  load_slice(0);
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      As[e >> 6][e & 63] = ra[u];
      Bs[e & 15][e >> 4] = rb[u];
    }
    __syncthreads();
    if (k0 + 16 < K) load_slice(k0 + 16);
    const int kc = min(16, K - k0);  // steps of 4 past kc would multiply zeros
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      if (k4 >= kc) break;
      const int kk = k4 + (l >> 4);
      cx<R> av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk][wi + 16 * a + (l & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][wj + 16 * b + (l & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = M::mac(bv[b].x, av[a].x, cr[a][b]);
          cr[a][b] = M::mac(-bv[b].y, av[a].y, cr[a][b]);
          ci[a][b] = M::mac(bv[b].y, av[a].x, ci[a][b]);
          ci[a][b] = M::mac(bv[b].x, av[a].y, ci[a][b]);
        }
    }
    __syncthreads();
    if constexpr (sizeof(R) != sizeof(double)) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            fr[a][b][v] += (double)cr[a][b][v];
            fi[a][b][v] += (double)ci[a][b][v];
          }
          cr[a][b] = acc_t{0, 0, 0, 0};
          ci[a][b] = acc_t{0, 0, 0, 0};
        }
    }
  }
  // block (a, b) holds rows wi + 16 a + (l & 15) of C and columns wj + 16 b + M::row(l, v)
  if constexpr (std::is_same<SubAt, std::nullptr_t>::value) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int li = wi + 16 * a + (l & 15), lj = wj + 16 * b + M::row(l, v);
          if (i0 + li < Mr && j0 + lj < Nc) {
            const double re = sizeof(R) == sizeof(double) ? (double)cr[a][b][v] : fr[a][b][v];
            const double im = sizeof(R) == sizeof(double) ? (double)ci[a][b][v] : fi[a][b][v];
            emit(li, lj, re, im);
          }
        }
  } else {
    (void)emit;
    // global (not flat) accesses, and no branches: elements outside the
    // product read and write a sink slot of this lane instead, so the 16
    // loads go out together and the stores need no wait on one another
    typedef __attribute__((address_space(1))) R* gptr;  // (real, imaginary) pairs
    const gptr sink = (gptr)(reinterpret_cast<R*>(rss_rmw_sink) + 2 * threadIdx.x);
    gptr p[2][2][4];
    R ore[2][2][4], oim[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int li = wi + 16 * a + (l & 15), lj = wj + 16 * b + M::row(l, v);
          p[a][b][v] = (i0 + li < Mr && j0 + lj < Nc) ? (gptr) reinterpret_cast<R*>(sub_at(li, lj)) : sink;
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          ore[a][b][v] = p[a][b][v][0];
          oim[a][b][v] = p[a][b][v][1];
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double re = sizeof(R) == sizeof(double) ? (double)cr[a][b][v] : fr[a][b][v];
          const double im = sizeof(R) == sizeof(double) ? (double)ci[a][b][v] : fi[a][b][v];
          p[a][b][v][0] = ore[a][b][v] - (R)(sub_scale * re);
          p[a][b][v][1] = oim[a][b][v] - (R)(sub_scale * im);
        }
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc<R>* desc, int tiles_m) {
  const GemmDesc<R> d = desc[blockIdx.x];
  const int tm = blockIdx.y % tiles_m, tn = blockIdx.y / tiles_m;
  const int i0 = tm * 64, j0 = tn * 64;
  if (i0 >= d.M || j0 >= d.N) return;
  const double sg = (double)d.sign;
  if (d.beta) {
    // C += sign A B, as C - (-sign) A B through the overlapped read-modify-write
    gemm_tile<R>(
        d.A, d.lda, d.B, d.ldb, d.M, d.N, d.K, i0, j0, [](int, int, double, double) {},
        [&](int li, int lj) { return d.C + (i0 + li) + (int64_t)(j0 + lj) * d.ldc; }, -sg);
  } else {
    gemm_tile<R>(d.A, d.lda, d.B, d.ldb, d.M, d.N, d.K, i0, j0, [&](int li, int lj, double re, double im) {
      d.C[(i0 + li) + (int64_t)(j0 + lj) * d.ldc] = cx<R>{(R)(sg * re), (R)(sg * im)};
    });
  }
}

// Schur update of one box (eq. e:step) as one product (three waves per SIMD:
// the tiles are latency-bound chains, and a third resident workgroup per CU
// covers more of them than the registers it takes cost; four spill):
//   [A_SS A_SN; A_NS A_NN] -= [X_SR; X_NR] Y,   Y = X_RR^{-1} [X_RS X_RN],
// rows and columns ordered [S; N_1 .. N_8] (Q = k + |N|).  Workgroup (slot, tile)
// computes a 64 x 64 tile of the Q x Q product and subtracts each element from
// the stencil block of its row box and column box.
template <class R>
__global__ __launch_bounds__(256, 3) void k_schur(const Prob<R>* probs, Phase<R> ph, int tiles_q) {
  __shared__ cx<R>* bp[9][9];
  __shared__ int ldr[9];
  __shared__ unsigned char rbk[64], cbk[64];
  __shared__ short rloc[64], cloc[64];
  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  const int Q = k + nN;
  const int i0 = (blockIdx.y % tiles_q) * 64, j0 = (blockIdx.y / tiles_q) * 64;
  if (r == 0 || i0 >= Q || j0 >= Q) return;
  int box[9], off[9], cnt[9];
  box[0] = b;
  off[0] = 0;
  cnt[0] = k;
  int o = k;
  int ncur[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) box[j + 1] = box_at(L, b, nb_dx(j), nb_dy(j));
#pragma unroll
  for (int j = 0; j < 8; ++j) ncur[j] = L.cur[box[j + 1] >= 0 ? box[j + 1] : b];  // loaded together
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    off[j + 1] = o;
    cnt[j + 1] = box[j + 1] >= 0 ? ncur[j] : 0;
    o += cnt[j + 1];
  }
  const int t = threadIdx.x;
  if (t < 81) {
    const int t1 = t / 9, t2 = t % 9;
    bp[t1][t2] = (box[t1] >= 0 && box[t2] >= 0) ? block_ptr(L, box[t1], box[t2]) : nullptr;
  }
  if (t < 9) ldr[t] = box[t] >= 0 ? L.n0[box[t]] : 0;
  if (t < 128) {
    // row (t < 64) or column (t >= 64) i0/j0 + (t & 63): its box and local index
    const int g = (t < 64 ? i0 : j0) + (t & 63);
    int q = 0;
    for (int u = 1; u < 9; ++u)
      if (cnt[u] > 0 && g >= off[u]) q = u;
    if (t < 64) {
      rbk[t] = (unsigned char)q;
      rloc[t] = (short)(g - off[q]);
    } else {
      cbk[t - 64] = (unsigned char)q;
      cloc[t - 64] = (short)(g - off[q]);
    }
  }
  __syncthreads();
  const cx<R>* XA = rec.F + rec.oXSNR[b];  // Q x r
  const cx<R>* YB = rec.F + rec.oY[b];     // r x Q
  gemm_tile<R>(XA, Q, YB, r, Q, Q, r, i0, j0, [](int, int, double, double) {}, [&](int li, int lj) {
    const int rb = rbk[li], cb = cbk[lj];
    return bp[rb][cb] + rloc[li] + (int64_t)cloc[lj] * ldr[rb];
  });
}

template <class R>
void launch_schur(const Prob<R>* probs, const Phase<R>& ph, int qmax, hipStream_t s) {
  if (ph.nbox == 0 || qmax <= 0) return;
  const int tq = (qmax + 63) / 64;
  hipLaunchKernelGGL(k_schur<R>, dim3(ph.nbox, tq * tq), dim3(256), 0, s, probs, ph, tq);
}

template <class R>
void launch_gemm(const GemmDesc<R>* desc, int ndesc, int max_m, int max_n, hipStream_t s) {
  if (ndesc == 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = (max_m + 63) / 64, tn = (max_n + 63) / 64;
  hipLaunchKernelGGL(k_gemm<R>, dim3(ndesc, tm * tn), dim3(256), 0, s, desc, tm);
}

// ---------------------------------------------------------------------------
// drop R: every stored block of B keeps only the skeleton rows / columns
// (in ascending order), and B's active ids shrink to S.
// ---------------------------------------------------------------------------
constexpr int COMPACT_PER = 8;

// rows of A (ld, ncols columns): row i <- row Sl[i] for i < k; columns independent
template <class R>
__device__ void compact_rows(cx<R>* A, int ld, const int* Sl, int k, int ncols) {
  constexpr int PER = COMPACT_PER;
  const int cw = max(1, (256 * PER) / max(k, 1));
  for (int c0 = 0; c0 < ncols; c0 += cw) {
    const int nc = min(cw, ncols - c0);
    cx<R> tmp[PER];
    int cnt = 0;
    for (int e = threadIdx.x; e < k * nc && cnt < PER; e += 256, ++cnt) {
      const int i = e % k, c = c0 + e / k;
      tmp[cnt] = A[Sl[i] + (int64_t)c * ld];
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < k * nc && cnt < PER; e += 256, ++cnt) {
      const int i = e % k, c = c0 + e / k;
      A[i + (int64_t)c * ld] = tmp[cnt];
    }
    __syncthreads();
  }
}

// columns of A (ld, nrows rows): column j <- column Sl[j] for j < k; rows independent
template <class R>
__device__ void compact_cols(cx<R>* A, int ld, const int* Sl, int k, int nrows) {
  constexpr int PER = COMPACT_PER;
  const int rw = max(1, (256 * PER) / max(k, 1));
  for (int i0 = 0; i0 < nrows; i0 += rw) {
    const int nr = min(rw, nrows - i0);
    cx<R> tmp[PER];
    int cnt = 0;
    for (int e = threadIdx.x; e < k * nr && cnt < PER; e += 256, ++cnt) {
      const int i = i0 + e % nr, j = e / nr;
      tmp[cnt] = A[i + (int64_t)Sl[j] * ld];
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < k * nr && cnt < PER; e += 256, ++cnt) {
      const int i = i0 + e % nr, j = e / nr;
      A[i + (int64_t)j * ld] = tmp[cnt];
    }
    __syncthreads();
  }
}

// B's active ids shrink to S and its size to k
template <class R>
__device__ void compact_ids(const Level<R>& L, int b, const int* Sl, int k) {
  int* gid = L.idx + L.ioff[b];
  for (int base = 0; base < k; base += 256) {
    const int i = base + threadIdx.x;
    const int v = i < k ? gid[Sl[i]] : 0;
    __syncthreads();
    if (i < k) gid[i] = v;
    __syncthreads();
  }
  if (threadIdx.x == 0) L.cur[b] = k;
}

// nine colours: workgroup (slot, s) handles the stencil pair s of the box,
// rows of A[b, b2] and columns of A[b2, b] (the diagonal block: rows, then
// columns, then the ids).  Boxes of one colour are 3 apart: no block is
// touched by two of them.
template <class R>
__global__ __launch_bounds__(256) void k_compact(const Prob<R>* probs, Phase<R> ph) {
  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int k = rec.k[b], r = rec.r[b];
  if (r == 0) return;
  const int s = blockIdx.y;
  const int b2 = box_at(L, b, s % 5 - 2, s / 5 - 2);
  if (b2 < 0) return;
  const int n0b = L.n0[b];
  const int* Sl = ph.Wi + ph.oI[slot];
  if (b2 != b) {
    const int c2 = L.cur[b2];
    compact_rows(block_ptr(L, b, b2), n0b, Sl, k, c2);
    compact_cols(block_ptr(L, b2, b), L.n0[b2], Sl, k, c2);
  } else {
    cx<R>* A = block_ptr(L, b, b);
    compact_rows(A, n0b, Sl, k, L.cur[b]);
    compact_cols(A, n0b, Sl, k, k);
    compact_ids(L, b, Sl, k);
  }
}

// four colours: boxes of one colour are 2 apart, so A[b, b2] of two such
// boxes has its rows dropped by one and its columns by the other.  Pass 0:
// rows of every A[b, .]; pass 1: columns of every A[., b]; the sizes and ids
// change only after both (k_compact_ids), so every pass reads the sizes the
// colour started with (rows beyond a new size are stale and never read).
template <class R>
__global__ __launch_bounds__(256) void k_compact_pass(const Prob<R>* probs, Phase<R> ph, int pass) {
  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  const int k = rec.k[b], r = rec.r[b];
  if (r == 0) return;
  const int s = blockIdx.y;
  const int b2 = box_at(L, b, s % 5 - 2, s / 5 - 2);
  if (b2 < 0) return;
  const int* Sl = ph.Wi + ph.oI[slot];
  if (pass == 0)
    compact_rows(block_ptr(L, b, b2), L.n0[b], Sl, k, L.cur[b2]);
  else
    compact_cols(block_ptr(L, b2, b), L.n0[b2], Sl, k, b2 == b ? k : L.cur[b2]);
}

template <class R>
__global__ __launch_bounds__(256) void k_compact_ids(const Prob<R>* probs, Phase<R> ph) {
  const int slot = blockIdx.x, b = ph.box[slot];
  const Level<R> L = probs[ph.prob[slot]].L;
  const Records<R> rec = probs[ph.prob[slot]].rec;
  if (rec.r[b] == 0) return;
  compact_ids(L, b, ph.Wi + ph.oI[slot], rec.k[b]);
}

template <class R>
void launch_compact(const Prob<R>* probs, const Phase<R>& ph, int colours, hipStream_t s) {
  if (ph.nbox == 0) return;
  if (colours != 4) {
    hipLaunchKernelGGL(k_compact<R>, dim3(ph.nbox, 25), dim3(256), 0, s, probs, ph);
    return;
  }
  hipLaunchKernelGGL(k_compact_pass<R>, dim3(ph.nbox, 25), dim3(256), 0, s, probs, ph, 0);
  hipLaunchKernelGGL(k_compact_pass<R>, dim3(ph.nbox, 25), dim3(256), 0, s, probs, ph, 1);
  hipLaunchKernelGGL(k_compact_ids<R>, dim3(ph.nbox), dim3(256), 0, s, probs, ph);
}

// ---------------------------------------------------------------------------
// merge (Sec. 2.5, Fig. f:merge): a block over the union of child skeletons,
// copied from the child blocks where the two children are within distance 2
// and evaluated fresh from the kernel otherwise (Thm. a:bm).
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_assemble_pairs(const PairDesc* pd, const ListEntry* lists,
                                                        int tiles_r, const Prob<R>* probs) {
  // the tile's 64 rows and 64 columns (list entry, coordinates, point scale)
  // and, for the Helmholtz kernel, the H0 table, staged in LDS
  __shared__ __align__(16) double stab[RSS_BESSEL_TAB];
  __shared__ double px[128], py[128], ps[128];
  __shared__ int pbox[128], pbx[128], pby[128], pn0[128], ploc[128], pgid[128];
  const PairDesc d = pd[blockIdx.x];
  const int tr = blockIdx.y % tiles_r, tc = blockIdx.y / tiles_r;
  const int i0 = tr * 64, j0 = tc * 64;
  if (i0 >= d.nr || j0 >= d.nc) return;
  const Level<R> child = probs[d.prob].L;
  const KParams kp = probs[d.prob].kp;
  const double* P = probs[d.prob].P;
  if (kp.kind == 1)
    for (int e = threadIdx.x; e < RSS_BESSEL_TAB; e += 256) stab[e] = rss_poly_jy[e];
  if (threadIdx.x < 128) {
    const int t = threadIdx.x & 63;
    const bool isrow = threadIdx.x < 64;
    const int k = (isrow ? i0 : j0) + t, kn = isrow ? d.nr : d.nc;
    if (k < kn) {
      const ListEntry le = (isrow ? lists + d.roff : lists + d.coff)[k];
      const double x = P[2 * le.gid], y = P[2 * le.gid + 1];
      pbox[threadIdx.x] = le.box;
      const int cnb = d.have_child ? child.nb : 1;  // child-grid coordinates of the box
      pbx[threadIdx.x] = le.box % cnb;
      pby[threadIdx.x] = le.box / cnb;
      pn0[threadIdx.x] = d.have_child ? child.n0[le.box] : 0;
      ploc[threadIdx.x] = le.local;
      pgid[threadIdx.x] = le.gid;
      px[threadIdx.x] = x;
      py[threadIdx.x] = y;
      ps[threadIdx.x] = point_scale(kp, x, y);
    }
  }
  __syncthreads();
  const double* tab = kp.kind == 1 ? (const double*)stab : rss_poly_jy;
  cx<R>* out = (cx<R>*)d.dst;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int li = e & 63, lj = e >> 6;
    const int i = i0 + li, j = j0 + lj;
    if (i >= d.nr || j >= d.nc) continue;
    const int cj = 64 + lj;
    cx<R> v;
    bool stored = false;
    if (d.have_child) {
      const int rb = pbox[li];
      const int dx = pbx[cj] - pbx[li];
      const int dy = pby[cj] - pby[li];
      if (abs(dx) <= 2 && abs(dy) <= 2) {
        const cx<R>* blk = child.A + child.boff[(int64_t)rb * 25 + slot_of(dx, dy)];
        v = blk[ploc[li] + (int64_t)ploc[cj] * pn0[li]];
        stored = true;
      }
    }
    if (!stored) {
      // the matrix entry of eq. e:aij, as entry() forms it, from the staged points
      cx<double> a;
      if (pgid[li] == pgid[cj]) {
        a = diag_entry(kp, ps[li]);
      } else {
        const cx<double> k = kernel_raw(kp, px[li], py[li], px[cj], py[cj], tab);
        double w = kp.weight;
        if (kp.bump) w *= ps[li] * ps[cj];
        a = cx<double>{w * k.x, w * k.y};
      }
      v = from_d<R>(a.x, a.y);
    }
    out[i + (int64_t)j * d.ld] = v;
    if (d.dstT) ((cx<R>*)d.dstT)[j + (int64_t)i * d.ldT] = v;
  }
}

template <class R>
void launch_assemble_pairs(const PairDesc* pd, int npairs, const ListEntry* lists, int max_r,
                           int max_c, const Prob<R>* child, hipStream_t s) {
  if (npairs == 0 || max_r <= 0 || max_c <= 0) return;
  const int tr = (max_r + 63) / 64, tc = (max_c + 63) / 64;
  hipLaunchKernelGGL(k_assemble_pairs<R>, dim3(npairs, tr * tc), dim3(256), 0, s, pd, lists, tr,
                     child);
}

// ---------------------------------------------------------------------------
// root: dense inverse by blocked Gauss-Jordan elimination with partial
// pivoting, in place in A, for all problems of a batch.  Per panel of NB
// columns [k0, k0 + NB): one workgroup per problem runs the NB elimination
// steps on the panel columns only (pivot search in the current column,
// interchange of whole rows, the Gauss-Jordan update of the panel); the
// elimination then reaches every other column X as one product,
//   X <- [X with the panel rows zeroed] + W X_P,
// W = the panel columns after the NB steps, X_P = the panel rows of X: one
// batched GEMM launch (matrix cores) per panel.  Finally the row interchanges
// are undone as column interchanges in reverse order, gathering into tmp.
// ---------------------------------------------------------------------------
constexpr int ROOT_NB = 32;
constexpr int ROOT_FEW = 8;  // batches up to this size use the unblocked form

template <class R>
__global__ __launch_bounds__(1024) void k_root_panel(const RootDesc<R>* rd, int k0, int* errflag) {
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  __shared__ cx<R> rowk[ROOT_NB];
  const RootDesc<R> d = rd[blockIdx.x];
  const int n = d.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) *d.gd = GemmDesc<R>{d.A, d.W, d.W, n, n, ROOT_NB, 0, 0, 0, 1, 1};  // no update
  if (k0 >= n) return;
  const int nbp = min(ROOT_NB, n - k0);
  cx<R>* A = d.A;
  cx<R>* Wt = d.W;                          // n x nbp (leading dimension n)
  cx<R>* Xp = Wt + (size_t)n * ROOT_NB;     // nbp x n (leading dimension ROOT_NB)
  cx<R>* cb = Xp + (size_t)ROOT_NB * n;     // column kk before the step
  for (int t = 0; t < nbp; ++t) {
    const int kk = k0 + t;
    // pivot: largest |A(i, kk)| over i >= kk, smallest i on ties
    double best = -1.0;
    int bi = n;
    for (int i = kk + threadIdx.x; i < n; i += NT) {
      const double v = abs2d(A[i + (int64_t)kk * n]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double v2 = __shfl_xor(best, o, 64);
      const int i2 = __shfl_xor(bi, o, 64);
      if (v2 > best || (v2 == best && i2 < bi)) {
        best = v2;
        bi = i2;
      }
    }
    if (lane == 0) {
      rv[wv] = best;
      ri[wv] = bi;
    }
    __syncthreads();
    best = rv[0];
    bi = ri[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (rv[w] > best || (rv[w] == best && ri[w] < bi)) {
        best = rv[w];
        bi = ri[w];
      }
    if (!(best > 0.0) || bi >= n) {
      if (threadIdx.x == 0) atomicOr(errflag, ERRF_SINGULAR);
      return;  // uniform
    }
    const int p = bi;
    if (threadIdx.x == 0) d.perm[kk] = p;
    if (p != kk)
      for (int j = threadIdx.x; j < n; j += NT) {
        const cx<R> a = A[kk + (int64_t)j * n];
        A[kk + (int64_t)j * n] = A[p + (int64_t)j * n];
        A[p + (int64_t)j * n] = a;
      }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) cb[i] = A[i + (int64_t)kk * n];
    if (threadIdx.x < nbp) rowk[threadIdx.x] = A[kk + (int64_t)(k0 + threadIdx.x) * n];
    __syncthreads();
    const cx<R> akk = rowk[t];
    const double dd = abs2d(akk);
    const cx<R> pinv{(R)(akk.x / dd), (R)(-akk.y / dd)};
    for (int e = threadIdx.x; e < n * nbp; e += NT) {
      const int jj = e / n, i = e - jj * n, j = k0 + jj;
      const cx<R> aik = cb[i], akj = rowk[jj];
      cx<R>* a = A + i + (int64_t)j * n;
      if (j == kk) *a = (i == kk) ? pinv : czero<R>() - aik * pinv;
      else *a = (i == kk) ? akj * pinv : *a - aik * pinv * akj;
    }
    __syncthreads();
  }
  // W, X_P (panel columns of X_P zero), and the panel rows of X cleared
  for (int e = threadIdx.x; e < n * nbp; e += NT) {
    const int jj = e / n, i = e - jj * n;
    Wt[i + (int64_t)jj * n] = A[i + (int64_t)(k0 + jj) * n];
  }
  for (int e = threadIdx.x; e < nbp * n; e += NT) {
    const int j = e / nbp, t = e - j * nbp;
    const bool panel = j >= k0 && j < k0 + nbp;
    cx<R>* a = A + (k0 + t) + (int64_t)j * n;
    Xp[t + (int64_t)j * ROOT_NB] = panel ? czero<R>() : *a;
    if (!panel) *a = czero<R>();
  }
  if (threadIdx.x == 0) *d.gd = GemmDesc<R>{A, Wt, Xp, n, n, ROOT_NB, n, n, nbp, 1, 1};
}

// Few problems: unblocked Gauss-Jordan, two pivot steps per launch for all of
// them (ping-pong buffers; each launch is bound by its chain of dependent
// loads: key, pivot, search column, second pivot row, tile); the first pivot of a
// launch is chosen by the launch that produces its column (packed |a| / index
// keys in W, atomicMax), the second by every workgroup of the launch itself.
// Pivot keys are zeroed and, for an odd number of launches (n + 1) / 2, A is
// copied to tmp first, so that the last launch writes A.
__host__ __device__ inline int root_launches(int n) { return (n + 1) / 2; }

template <class R>
__global__ __launch_bounds__(256) void k_root_prep(const RootDesc<R>* rd) {
  const RootDesc<R> d = rd[blockIdx.y];
  const int n = d.n;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(d.W);
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t e = e0; e < n; e += (int64_t)gridDim.x * 256) keys[e] = 0ull;
  if (root_launches(n) & 1)
    for (int64_t e = e0; e < (int64_t)n * n; e += (int64_t)gridDim.x * 256) d.tmp[e] = d.A[e];
}

__device__ __forceinline__ unsigned long long pivkey(double a2, int i) {
  const float f = (float)sqrt(a2);
  return ((unsigned long long)__float_as_uint(f) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
}

template <class R>
__global__ __launch_bounds__(256) void k_root_pivot0(const RootDesc<R>* rd) {
  __shared__ unsigned long long red[256];
  const RootDesc<R> d = rd[blockIdx.x];
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(d.W);
  unsigned long long best = 0;
  for (int i = threadIdx.x; i < d.n; i += 256) {
    const unsigned long long kk = pivkey(abs2d(d.A[i]), i);
    best = kk > best ? kk : best;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) keys[0] = red[0];
}

// Pivot steps kk and kk + 1 (only kk when kk + 1 == n) on a 32 x 32 tile.
// Step kk with pivot row p (its key from the previous launch) takes src to
//   v1(r, j) = src(p, j) / a                        r = kk (j != kk; 1 / a at j = kk)
//            = src(s, j) - src(s, kk) / a src(p, j)  r != kk, s = r with rows kk, p exchanged
// (-src(s, kk) / a at j = kk), a = src(p, kk); step kk + 1 applies the same
// rule to v1 with pivot p2 = the row r >= kk + 1 of largest |v1(r, kk + 1)|
// (smallest r on ties), which every workgroup forms from src for itself.  The
// workgroups holding column kk + 2 publish its pivot key for the next launch.
template <class R>
__global__ __launch_bounds__(256) void k_root_gj(const RootDesc<R>* rd, int kk, int* errflag) {
  __shared__ unsigned long long wred[4];
  __shared__ cx<R> rowp2[32];
  const RootDesc<R> d = rd[blockIdx.z];
  const int n = d.n;
  if (kk >= n) return;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  if (i0 >= n || j0 >= n) return;
  const bool fromtmp = ((kk / 2 + root_launches(n)) & 1) != 0;
  const cx<R>* src = fromtmp ? d.tmp : d.A;
  cx<R>* dst = fromtmp ? d.A : d.tmp;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(d.W);
  const bool first = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  const unsigned long long key = keys[kk];
  const int p = (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
  if (key == 0ull || p < kk || p >= n) {  // no pivot recorded (an earlier step was singular)
    if (first) atomicOr(errflag, ERRF_SINGULAR);
    return;
  }
  const cx<R> akk = src[p + (int64_t)kk * n];
  const double dd = abs2d(akk);
  if (dd == 0.0) {
    if (first) atomicOr(errflag, ERRF_SINGULAR);
    return;
  }
  const cx<R> pinv{(R)(akk.x / dd), (R)(-akk.y / dd)};
  // entry (r, j) after step kk
  auto v1 = [&](int r, int j) -> cx<R> {
    if (r == kk) return j == kk ? pinv : src[p + (int64_t)j * n] * pinv;
    const int sr = (r == p) ? kk : r;
    const cx<R> aik = src[sr + (int64_t)kk * n];
    if (j == kk) return czero<R>() - aik * pinv;
    return src[sr + (int64_t)j * n] - aik * pinv * src[p + (int64_t)j * n];
  };
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool two = kk + 1 < n;
  const int k2 = kk + 1;
  // this thread: row i, columns j0 + cg + 8 m.  The loads that every row
  // other than k2 and p2 needs are issued before the second pivot is known.
  const int i = i0 + (lane & 31), cg = (int)threadIdx.x >> 5;
  const int sr = (i == p) ? kk : i;  // source row of row i in step kk
  const bool rv = i < n && i != kk;
  cx<R> s_j[4], p_j[4];
  const cx<R> aik_i = rv ? src[sr + (int64_t)kk * n] : czero<R>();
  const cx<R> s_k2 = rv && two ? src[sr + (int64_t)k2 * n] : czero<R>();
  const cx<R> p_k2 = two ? src[p + (int64_t)k2 * n] : czero<R>();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = j0 + cg + 8 * m;
    s_j[m] = (rv && j < n) ? src[sr + (int64_t)j * n] : czero<R>();
    p_j[m] = (i < n && j < n) ? src[p + (int64_t)j * n] : czero<R>();
  }
  int p2 = 0;
  cx<R> pinv2 = czero<R>();
  if (two) {
    unsigned long long best = 0;
    for (int r = k2 + (int)threadIdx.x; r < n; r += 256) {
      const unsigned long long kq = pivkey(abs2d(v1(r, k2)), r);
      best = kq > best ? kq : best;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned hi = __shfl_xor((unsigned)(best >> 32), o, 64), lo = __shfl_xor((unsigned)best, o, 64);
      const unsigned long long b2 = ((unsigned long long)hi << 32) | lo;
      best = b2 > best ? b2 : best;
    }
    if (lane == 0) wred[wv] = best;
    __syncthreads();
    best = max(max(wred[0], wred[1]), max(wred[2], wred[3]));
    p2 = (int)(0xFFFFFFFFu - (unsigned)(best & 0xFFFFFFFFull));
    if (best == 0ull || p2 <= kk || p2 >= n) {
      if (first) atomicOr(errflag, ERRF_SINGULAR);
      return;  // uniform: every workgroup takes the same decision
    }
    const cx<R> a2 = v1(p2, k2);
    const double d2 = abs2d(a2);
    if (d2 == 0.0) {
      if (first) atomicOr(errflag, ERRF_SINGULAR);
      return;
    }
    pinv2 = cx<R>{(R)(a2.x / d2), (R)(-a2.y / d2)};
  }
  if (threadIdx.x < 32) {
    const int j = j0 + (int)threadIdx.x;
    if (j < n && two) rowp2[threadIdx.x] = v1(p2, j);
  }
  if (first) {
    d.perm[kk] = p;
    if (two) d.perm[kk + 1] = p2;
  }
  __syncthreads();
  // rows k2 and p2 exchange in step kk + 1: those two rows load afresh
  const bool plain = !two || (i != k2 && i != p2);
  const int s2 = !two ? i : (i == k2 ? p2 : (i == p2 ? k2 : i));
  // entry (i, j) after step kk from the preloaded values (i != kk)
  auto v1pre = [&](int m, int j) -> cx<R> {
    if (j == kk) return czero<R>() - aik_i * pinv;
    return s_j[m] - aik_i * pinv * p_j[m];
  };
  cx<R> a = czero<R>();
  if (two && i < n) {
    if (!plain) a = v1(s2, k2);
    else if (i == kk) a = p_k2 * pinv;
    else a = s_k2 - aik_i * pinv * p_k2;
  }
  unsigned long long nbest = 0;
  const int jn = kk + 2;  // the column whose pivot the next launch needs
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = j0 + cg + 8 * m;
    if (i >= n || j >= n) continue;
    // v1(s2, j)
    cx<R> w;
    if (!plain) w = v1(s2, j);
    else if (i == kk) w = (j == kk) ? pinv : p_j[m] * pinv;
    else w = v1pre(m, j);
    cx<R> v;
    if (!two) {
      v = w;
    } else if (i == k2) {
      v = (j == k2) ? pinv2 : rowp2[j - j0] * pinv2;
    } else {
      v = (j == k2) ? czero<R>() - a * pinv2 : w - a * pinv2 * rowp2[j - j0];
    }
    dst[i + (int64_t)j * n] = v;
    if (j == jn && i >= jn) nbest = pivkey(abs2d(v), i);
  }
  // the wave holding column kk + 2 (in one half of its lanes) posts its key
  if (two && jn < n && jn >= j0 && jn < j0 + 32 && (((jn - j0) & 7) >> 1) == wv) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned hi = __shfl_xor((unsigned)(nbest >> 32), o, 64), lo = __shfl_xor((unsigned)nbest, o, 64);
      const unsigned long long b2 = ((unsigned long long)hi << 32) | lo;
      nbest = b2 > nbest ? b2 : nbest;
    }
    if (lane == 0 && nbest) atomicMax(keys + jn, nbest);
  }
}

// column interchanges of the row interchanges, in reverse order
template <class R>
__global__ __launch_bounds__(64) void k_root_finish(const RootDesc<R>* rd) {
  const RootDesc<R> d = rd[blockIdx.y];
  const int n = d.n;
  int* cp = d.perm + n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) cp[j] = j;
    for (int kk = n - 1; kk >= 0; --kk) {
      int p = d.perm[kk];
      if (p < 0 || p >= n) p = kk;
      const int t = cp[kk];
      cp[kk] = cp[p];
      cp[p] = t;
    }
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_root_gather(const RootDesc<R>* rd) {
  const RootDesc<R> d = rd[blockIdx.y];
  const int n = d.n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  d.tmp[e] = d.A[i + (int64_t)d.perm[n + j] * n];
}

// gd: one GemmDesc per problem (device); the inverse ends in tmp
template <class R>
void launch_root_inverse(const RootDesc<R>* rd, int nprob, int nmax, GemmDesc<R>* gd, int* errflag,
                         hipStream_t s) {
  if (nprob == 0 || nmax == 0) return;
  if (nprob <= ROOT_FEW) {
    const int64_t tot = (int64_t)nmax * nmax;
    hipLaunchKernelGGL(k_root_prep<R>, dim3((unsigned)std::min<int64_t>(4096, (tot + 255) / 256), nprob), dim3(256),
                       0, s, rd);
    hipLaunchKernelGGL(k_root_pivot0<R>, dim3(nprob), dim3(256), 0, s, rd);
    const int t = (nmax + 31) / 32;
    for (int kk = 0; kk < nmax; kk += 2)
      hipLaunchKernelGGL(k_root_gj<R>, dim3(t, t, nprob), dim3(256), 0, s, rd, kk, errflag);
  } else {
    for (int k0 = 0; k0 < nmax; k0 += ROOT_NB) {
      hipLaunchKernelGGL(k_root_panel<R>, dim3(nprob), dim3(1024), 0, s, rd, k0, errflag);
      launch_gemm<R>(gd, nprob, nmax, nmax, s);
    }
  }
  hipLaunchKernelGGL(k_root_finish<R>, dim3(1, nprob), dim3(64), 0, s, rd);
  const int64_t tot = (int64_t)nmax * nmax;
  hipLaunchKernelGGL(k_root_gather<R>, dim3((unsigned)((tot + 255) / 256), nprob), dim3(256), 0, s,
                     rd);
}

size_t root_work_elems(int n) { return (size_t)2 * n * ROOT_NB + (size_t)n; }

// ---------------------------------------------------------------------------
// solve sweeps (Sec. 2.6)
//  forward : z_R -= T^* z_S;  w = X_RR^{-1} z_R;  z_{S,N} -= [X_SR; X_NR] w
//  backward: x_R = X_RR^{-1} z_R - Y z_{S,N};  z_S -= T x_R;  z_R = x_R
// One workgroup per (box, group of up to SNC right-hand sides).  The sweeps
// stream small factor blocks and are bound by memory latency: each product
// gives every thread a task (row a, slice p of the summation index) that
// loads SU entries of its row at once, coalesced across the lanes of a wave,
// and uses each for all columns of the group (kept in registers).  Products
// with few rows split the summation over P = 256 / rows slices and reduce the
// slices in a fixed order through LDS.  Right-hand-side panels sit in LDS,
// row-major with stride sld = group + 1.
// ---------------------------------------------------------------------------
constexpr int SNC = 16;  // most right-hand sides per workgroup (registers per thread)
constexpr int SU = 16;   // factor entries loaded per thread per round
constexpr size_t SOLVE_LDS = 96 * 1024;
constexpr int SRED = 256;  // rows of the slice-reduction buffer

// right-hand sides per workgroup so that both sweeps' LDS fits the budget
// (0: not even one fits)
template <class R>
int solve_group(int kmax, int rmax, int nrhs) {
  const size_t rows = (size_t)std::max(kmax + 2 * rmax, 2 * rmax + 16) + SRED;
  for (int g = std::min(SNC, std::max(nrhs, 1)); g >= 1; --g)
    if (rows * (g + 1) * sizeof(cx<R>) <= SOLVE_LDS) return g;
  return 0;
}

template <class R>
__device__ __forceinline__ void zero_acc(cx<R> (&acc)[SNC]) {
#pragma unroll
  for (int c = 0; c < SNC; ++c) acc[c] = czero<R>();
}

// acc[c] += sum op(A)(a, s) Bz[(s - s_lo) sld + c] over the slice p of P of
// s in [s_lo, s_hi) (rounds of SU consecutive s, dealt round-robin);
// op(A)(a, s) = A[a + s lda], or conj(A[s + a lda]) when CT
template <class R, bool CT>
__device__ __forceinline__ void mm_slice(const cx<R>* __restrict__ A, int64_t lda, int a, int s_lo,
                                         int s_hi, int p, int P, const cx<R>* Bz, int sld, int nc,
                                         cx<R> (&acc)[SNC]) {
  for (int s0 = s_lo + p * SU; s0 < s_hi; s0 += P * SU) {
    cx<R> x[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int s = s0 + u;
      if (s < s_hi) x[u] = CT ? conj(A[s + (int64_t)a * lda]) : A[a + (int64_t)s * lda];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      if (s0 + u < s_hi) {
        const cx<R>* b = Bz + (s0 + u - s_lo) * sld;
#pragma unroll
        for (int c = 0; c < SNC; ++c)
          if (c < nc) fma_(acc[c], x[u], b[c]);
      }
    }
  }
}

// row a of op(A) Bz over s in [s_lo, s_hi) for every a < M, handed to
// emit(a, v) with v[c] for c < nc exactly once per row.  All threads of the
// workgroup call it (it synchronizes when M <= 128).  red: SRED * sld entries.
template <class R, bool CT, class Emit>
__device__ __forceinline__ void blk_mm(const cx<R>* __restrict__ A, int64_t lda, int M, int s_lo,
                                       int s_hi, const cx<R>* Bz, int sld, int nc, cx<R>* red,
                                       Emit emit) {
  if (M <= 0) return;
  const int Mb = M < 256 ? M : 256;
  const int P = 256 / Mb;
  const int t = threadIdx.x;
  cx<R> acc[SNC];
  for (int m0 = 0; m0 < M; m0 += Mb) {
    const int i = t % Mb, p = t / Mb, a = m0 + i;
    const bool act = p < P && a < M;
    zero_acc(acc);
    if (act) mm_slice<R, CT>(A, lda, a, s_lo, s_hi, p, P, Bz, sld, nc, acc);
    if (P == 1) {
      if (act) emit(a, acc);
    } else {
      if (act) {
#pragma unroll
        for (int c = 0; c < SNC; ++c)
          if (c < nc) red[(p * Mb + i) * sld + c] = acc[c];
      }
      __syncthreads();
      // slices summed in a fixed order into the rows of slice 0
      for (int e = t; e < Mb * nc; e += 256) {
        const int ii = e % Mb, c = e / Mb;
        cx<R> v = red[ii * sld + c];
        for (int q = 1; q < P; ++q) v = v + red[(q * Mb + ii) * sld + c];
        red[ii * sld + c] = v;
      }
      __syncthreads();
      if (t < Mb) {
#pragma unroll
        for (int c = 0; c < SNC; ++c) acc[c] = c < nc ? red[t * sld + c] : czero<R>();
        emit(m0 + t, acc);
      }
      __syncthreads();
    }
  }
}

// z[g + (c0 + c) ldz] -= v[c] for c < nc: every load before any store
template <class R>
__device__ __forceinline__ void sub_row(cx<R>* z, int64_t ldz, int64_t g, int c0, int nc,
                                        const cx<R> (&v)[SNC]) {
  cx<R> o[SNC];
  cx<R>* p = z + g + (int64_t)c0 * ldz;
#pragma unroll
  for (int c = 0; c < SNC; ++c)
    if (c < nc) o[c] = p[c * ldz];
#pragma unroll
  for (int c = 0; c < SNC; ++c)
    if (c < nc) p[c * ldz] = o[c] - v[c];
}

// z[g + (c0 + c) ldz] -= v[c] for c < nc by atomic adds (the four-colour
// schedule's forward sweep: boxes of a phase share neighbours; hipMalloc
// memory is coarse-grained, so the hardware float atomics apply)
template <class R>
__device__ __forceinline__ void sub_row_atomic(cx<R>* z, int64_t ldz, int64_t g, int c0, int nc,
                                               const cx<R> (&v)[SNC]) {
  R* p = reinterpret_cast<R*>(z + g + (int64_t)c0 * ldz);
#pragma unroll
  for (int c = 0; c < SNC; ++c)
    if (c < nc) {
      unsafeAtomicAdd(p + 2 * c * ldz, -v[c].x);
      unsafeAtomicAdd(p + 2 * c * ldz + 1, -v[c].y);
    }
}

// LDS panel P[i * sld + c] = z[g(i) + (c0 + c) ldz] for i < n, c < nc, eight
// loads in flight per thread
template <class R, class Idx>
__device__ __forceinline__ void gather(cx<R>* P, int sld, const cx<R>* z, int64_t ldz, int c0, int n,
                                       int nc, Idx g) {
  constexpr int GU = 8;
  const int tot = n * nc;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 256 * GU) {
    cx<R> v[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = e0 + 256 * u;
      if (e < tot) v[u] = z[g(e % n) + (int64_t)(c0 + e / n) * ldz];
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = e0 + 256 * u;
      if (e < tot) P[(e % n) * sld + e / n] = v[u];
    }
  }
}

// Slices per box for the two wide products of a phase ([X_SR; X_NR] w by
// rows, Y z_{S,N} by columns): enough workgroups for the whole chip when a
// colour holds few boxes.
int solve_slices(int nbox, int qmax) {
  int S = (512 + nbox - 1) / std::max(nbox, 1);
  S = std::min(S, std::max(1, (qmax + 47) / 48));
  return std::max(S, 1);
}

template <class R>
size_t solve_work_elems(int nbox, int rmax, int S, int nrhs) {
  return (size_t)nbox * S * rmax * nrhs;
}

// forward, part 1 (one workgroup per box and column group):
// z_R -= T^* z_S;  w = X_RR^{-1} z_R -> W[slot];  z_R written back
template <class R>
__global__ __launch_bounds__(256) void k_solve_fwd_a(const SolveProb<R>* sp, Phase<R> ph, int kmax,
                                                     int rmax, int ncg, cx<R>* W, int ldw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* zS = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* zR = zS + (int64_t)kmax * sld;
  cx<R>* red = zR + (int64_t)rmax * sld;
  const int slot = blockIdx.x, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int* gS = rec.G + rec.oS[b];
  const int* gR = rec.G + rec.oR[b];
  const cx<R>* T = rec.F + rec.oT[b];
  const cx<R>* Xi = rec.F + rec.oXi[b];
  gather(zS, sld, z, ldz, c0, k, nc, [&](int i) { return gS[i]; });
  gather(zR, sld, z, ldz, c0, r, nc, [&](int i) { return gR[i]; });
  __syncthreads();
  blk_mm<R, true>(T, k, r, 0, k, zS, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) zR[a * sld + c] = zR[a * sld + c] - v[c];
  });
  __syncthreads();
  cx<R>* Wb = W + (int64_t)slot * rmax * ldw + c0;
  blk_mm<R, false>(Xi, r, r, 0, r, zR, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) Wb[(int64_t)a * ldw + c] = v[c];
  });
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    z[gR[a] + (int64_t)(c0 + c) * ldz] = zR[a * sld + c];
  }
}

// forward in one workgroup per box and column group (the fused tile):
// z_R -= T^* z_S;  w = X_RR^{-1} z_R kept in LDS;  z_R written back;
// z_{S,N} -= [X_SR; X_NR] w.  Same arithmetic as parts 1 and 2 with one slice.
template <class R>
__global__ __launch_bounds__(256) void k_solve_fwd_fused(const SolveProb<R>* sp, Phase<R> ph, int kmax,
                                                         int rmax, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* zS = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* zR = zS + (int64_t)kmax * sld;
  cx<R>* red = zR + (int64_t)rmax * sld;
  cx<R>* w = red + (int64_t)SRED * sld;
  const int slot = blockIdx.x, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int* gS = rec.G + rec.oS[b];
  const int* gR = rec.G + rec.oR[b];
  const int* gN = rec.G + rec.oN[b];
  const cx<R>* T = rec.F + rec.oT[b];
  const cx<R>* Xi = rec.F + rec.oXi[b];
  const cx<R>* XS = rec.F + rec.oXSNR[b];
  gather(zS, sld, z, ldz, c0, k, nc, [&](int i) { return gS[i]; });
  gather(zR, sld, z, ldz, c0, r, nc, [&](int i) { return gR[i]; });
  __syncthreads();
  blk_mm<R, true>(T, k, r, 0, k, zS, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) zR[a * sld + c] = zR[a * sld + c] - v[c];
  });
  __syncthreads();
  blk_mm<R, false>(Xi, r, r, 0, r, zR, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) w[a * sld + c] = v[c];
  });
  __syncthreads();
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    z[gR[a] + (int64_t)(c0 + c) * ldz] = zR[a * sld + c];
  }
  const int q = k + nN;
  const bool at = ph.atomic_nbr != 0;
  blk_mm<R, false>(XS, q, q, 0, r, w, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
    if (a >= k && at)
      sub_row_atomic(z, ldz, gN[a - k], c0, nc, v);
    else
      sub_row(z, ldz, a < k ? gS[a] : gN[a - k], c0, nc, v);
  });
}

// forward, part 2 (S workgroups per box, each a slice of rows):
// z_{S,N} -= [X_SR; X_NR] w
template <class R>
__global__ __launch_bounds__(256) void k_solve_fwd_b(const SolveProb<R>* sp, Phase<R> ph, int rmax,
                                                     int ncg, int S, const cx<R>* W, int ldw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* w = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* red = w + (int64_t)rmax * sld;
  const int slot = blockIdx.x / S, j = blockIdx.x % S, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int q = k + nN, qs = (q + S - 1) / S, a_lo = j * qs, a_hi = min(q, a_lo + qs);
  if (a_lo >= a_hi) return;
  const int* gS = rec.G + rec.oS[b];
  const int* gN = rec.G + rec.oN[b];
  const cx<R>* XS = rec.F + rec.oXSNR[b];
  const cx<R>* Wb = W + (int64_t)slot * rmax * ldw + c0;
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    w[a * sld + c] = Wb[(int64_t)a * ldw + c];
  }
  __syncthreads();
  const bool at = ph.atomic_nbr != 0;
  blk_mm<R, false>(XS + a_lo, q, a_hi - a_lo, 0, r, w, sld, nc, red,
                   [&](int a, const cx<R>(&v)[SNC]) {
                     const int row = a_lo + a;
                     if (row >= k && at)
                       sub_row_atomic(z, ldz, gN[row - k], c0, nc, v);
                     else
                       sub_row(z, ldz, row < k ? gS[row] : gN[row - k], c0, nc, v);
                   });
}

template <class R>
void launch_solve_fwd(const SolveProb<R>* sp, const Phase<R>& ph, int nrhs, int kmax, int rmax,
                      int qmax, SolveTile tile, cx<R>* W, hipStream_t s) {
  (void)qmax;
  const int ncg = tile.ncg, S = tile.S;
  if (ph.nbox == 0 || ncg <= 0 || S <= 0) return;  // the caller validates the tile
  const size_t row = (size_t)(ncg + 1) * sizeof(cx<R>);
  const dim3 groups((nrhs + ncg - 1) / ncg);
  if (tile.fused) {
    hipLaunchKernelGGL(k_solve_fwd_fused<R>, dim3(ph.nbox, groups.x), dim3(256),
                       (size_t)(kmax + 2 * rmax + SRED) * row, s, sp, ph, kmax, rmax, ncg);
    return;
  }
  hipLaunchKernelGGL(k_solve_fwd_a<R>, dim3(ph.nbox, groups.x), dim3(256),
                     (size_t)(kmax + rmax + SRED) * row, s, sp, ph, kmax, rmax, ncg, W, nrhs);
  hipLaunchKernelGGL(k_solve_fwd_b<R>, dim3(ph.nbox * S, groups.x), dim3(256),
                     (size_t)(rmax + SRED) * row, s, sp, ph, rmax, ncg, S, (const cx<R>*)W, nrhs);
}

// backward, part 1 (S workgroups per box, each a slice of the columns of Y):
// W[slot, j] = Y[:, slice j] z_{S,N}[slice j]
template <class R>
__global__ __launch_bounds__(256) void k_solve_bwd_a(const SolveProb<R>* sp, Phase<R> ph, int rmax,
                                                     int chunk, int ncg, int S, cx<R>* W, int ldw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* xp = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* red = xp + (int64_t)rmax * sld;
  cx<R>* zq = red + (int64_t)SRED * sld;  // chunk rows of z_{S,N}
  const int slot = blockIdx.x / S, j = blockIdx.x % S, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int q = k + nN, qs = (q + S - 1) / S, s_lo = min(q, j * qs), s_hi = min(q, s_lo + qs);
  const int* gS = rec.G + rec.oS[b];
  const int* gN = rec.G + rec.oN[b];
  const cx<R>* Y = rec.F + rec.oY[b];
  for (int e = threadIdx.x; e < r * sld; e += 256) xp[e] = czero<R>();
  for (int q0 = s_lo; q0 < s_hi; q0 += chunk) {
    const int nq = min(chunk, s_hi - q0);
    __syncthreads();
    gather(zq, sld, z, ldz, c0, nq, nc,
           [&](int i) { return (q0 + i) < k ? gS[q0 + i] : gN[q0 + i - k]; });
    __syncthreads();
    blk_mm<R, false>(Y, r, r, q0, q0 + nq, zq, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
      for (int c = 0; c < SNC; ++c)
        if (c < nc) xp[a * sld + c] = xp[a * sld + c] + v[c];
    });
  }
  __syncthreads();
  cx<R>* Wb = W + ((int64_t)slot * S + j) * rmax * ldw + c0;
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    Wb[(int64_t)a * ldw + c] = xp[a * sld + c];
  }
}

// backward, part 2 (one workgroup per box and column group):
// x_R = X_RR^{-1} z_R - sum_j W[slot, j];  z_S -= T x_R;  z_R = x_R
template <class R>
__global__ __launch_bounds__(256) void k_solve_bwd_b(const SolveProb<R>* sp, Phase<R> ph, int rmax,
                                                     int ncg, int S, const cx<R>* W, int ldw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* zR = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* xR = zR + (int64_t)rmax * sld;
  cx<R>* red = xR + (int64_t)rmax * sld;
  const int slot = blockIdx.x, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int* gS = rec.G + rec.oS[b];
  const int* gR = rec.G + rec.oR[b];
  const cx<R>* T = rec.F + rec.oT[b];
  const cx<R>* Xi = rec.F + rec.oXi[b];
  gather(zR, sld, z, ldz, c0, r, nc, [&](int i) { return gR[i]; });
  __syncthreads();
  blk_mm<R, false>(Xi, r, r, 0, r, zR, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) xR[a * sld + c] = v[c];
  });
  __syncthreads();
  const cx<R>* Wb = W + (int64_t)slot * S * rmax * ldw + c0;
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    cx<R> v = xR[a * sld + c];
    const cx<R>* wp = Wb + (int64_t)a * ldw + c;
    const int64_t js = (int64_t)rmax * ldw;
    // slices in order, eight loads in flight
    for (int j0 = 0; j0 < S; j0 += 8) {
      cx<R> t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < S) t[u] = wp[(j0 + u) * js];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < S) v = v - t[u];
    }
    xR[a * sld + c] = v;
  }
  __syncthreads();
  blk_mm<R, false>(T, k, k, 0, r, xR, sld, nc, red,
                   [&](int a, const cx<R>(&v)[SNC]) { sub_row(z, ldz, gS[a], c0, nc, v); });
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    z[gR[a] + (int64_t)(c0 + c) * ldz] = xR[a * sld + c];
  }
}

// backward in one workgroup per box and column group (the fused tile):
// p = Y z_{S,N} (chunks of z_{S,N} in LDS, summed in chunk order);
// x_R = X_RR^{-1} z_R - p;  z_S -= T x_R;  z_R = x_R.  Same arithmetic as
// parts 1 and 2 with one slice.
template <class R>
__global__ __launch_bounds__(256) void k_solve_bwd_fused(const SolveProb<R>* sp, Phase<R> ph, int rmax,
                                                         int chunk, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sld = ncg + 1;
  cx<R>* xp = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* red = xp + (int64_t)rmax * sld;
  cx<R>* zq = red + (int64_t)SRED * sld;  // chunk rows of z_{S,N}; then z_R and x_R
  cx<R>* zR = zq;
  cx<R>* xR = zq + (int64_t)rmax * sld;
  const int slot = blockIdx.x, b = ph.box[slot];
  const SolveProb<R> pr = sp[ph.prob[slot]];
  const Records<R>& rec = pr.rec;
  cx<R>* z = pr.z;
  const int64_t ldz = pr.ldz;
  const int k = rec.k[b], r = rec.r[b], nN = rec.nN[b];
  if (r == 0) return;
  const int c0 = blockIdx.y * ncg;
  if (c0 >= pr.nrhs) return;
  const int nc = min(ncg, pr.nrhs - c0);
  const int q = k + nN;
  const int* gS = rec.G + rec.oS[b];
  const int* gR = rec.G + rec.oR[b];
  const int* gN = rec.G + rec.oN[b];
  const cx<R>* Y = rec.F + rec.oY[b];
  const cx<R>* T = rec.F + rec.oT[b];
  const cx<R>* Xi = rec.F + rec.oXi[b];
  for (int e = threadIdx.x; e < r * sld; e += 256) xp[e] = czero<R>();
  for (int q0 = 0; q0 < q; q0 += chunk) {
    const int nq = min(chunk, q - q0);
    __syncthreads();
    gather(zq, sld, z, ldz, c0, nq, nc,
           [&](int i) { return (q0 + i) < k ? gS[q0 + i] : gN[q0 + i - k]; });
    __syncthreads();
    blk_mm<R, false>(Y, r, r, q0, q0 + nq, zq, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
      for (int c = 0; c < SNC; ++c)
        if (c < nc) xp[a * sld + c] = xp[a * sld + c] + v[c];
    });
  }
  __syncthreads();
  gather(zR, sld, z, ldz, c0, r, nc, [&](int i) { return gR[i]; });
  __syncthreads();
  blk_mm<R, false>(Xi, r, r, 0, r, zR, sld, nc, red, [&](int a, const cx<R>(&v)[SNC]) {
#pragma unroll
    for (int c = 0; c < SNC; ++c)
      if (c < nc) xR[a * sld + c] = v[c] - xp[a * sld + c];
  });
  __syncthreads();
  blk_mm<R, false>(T, k, k, 0, r, xR, sld, nc, red,
                   [&](int a, const cx<R>(&v)[SNC]) { sub_row(z, ldz, gS[a], c0, nc, v); });
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    z[gR[a] + (int64_t)(c0 + c) * ldz] = xR[a * sld + c];
  }
}

// LDS rows (times ncg + 1 entries) of the backward kernels for a level: the
// chunk of z_{S,N} staged at once, and whether the fused kernel fits
template <class R>
static int bwd_chunk(int rmax, int qmax, int S, size_t row) {
  const int qs = (qmax + S - 1) / S;
  return (int)std::min<size_t>(std::max(qs, 16), SOLVE_LDS / row - (size_t)rmax - SRED);
}

template <class R>
bool solve_fused_fits(int kmax, int rmax, int ncg) {
  const size_t row = (size_t)(ncg + 1) * sizeof(cx<R>);
  return (size_t)(kmax + 2 * rmax + SRED) * row <= SOLVE_LDS &&
         (size_t)(3 * rmax + SRED) * row <= SOLVE_LDS;
}

template <class R>
void launch_solve_bwd(const SolveProb<R>* sp, const Phase<R>& ph, int nrhs, int kmax, int rmax,
                      int qmax, SolveTile tile, cx<R>* W, hipStream_t s) {
  (void)kmax;
  const int ncg = tile.ncg, S = tile.S;
  if (ph.nbox == 0 || ncg <= 0 || S <= 0) return;  // the caller validates the tile
  const size_t row = (size_t)(ncg + 1) * sizeof(cx<R>);
  const dim3 groups((nrhs + ncg - 1) / ncg);
  // z_{S,N} chunk: one slice's rows if they fit, else what is left of the budget (>= 16 rows)
  const int chunk = bwd_chunk<R>(rmax, qmax, tile.fused ? 1 : S, row);
  if (tile.fused) {
    const int u = std::max(chunk, 2 * rmax);  // the chunk, later z_R and x_R
    hipLaunchKernelGGL(k_solve_bwd_fused<R>, dim3(ph.nbox, groups.x), dim3(256),
                       (size_t)(rmax + SRED + u) * row, s, sp, ph, rmax, chunk, ncg);
    return;
  }
  hipLaunchKernelGGL(k_solve_bwd_a<R>, dim3(ph.nbox * S, groups.x), dim3(256),
                     (size_t)(rmax + SRED + chunk) * row, s, sp, ph, rmax, chunk, ncg, S, W, nrhs);
  hipLaunchKernelGGL(k_solve_bwd_b<R>, dim3(ph.nbox, groups.x), dim3(256),
                     (size_t)(2 * rmax + SRED) * row, s, sp, ph, rmax, ncg, S, (const cx<R>*)W,
                     nrhs);
}

// root apply for a batch: gather z[ids] -> ws, ws2 = Ainv ws (GEMM), scatter back
template <class R>
__global__ void k_root_gather_rhs(const RootApply<R>* ra, GemmDesc<R>* desc) {
  const RootApply<R> d = ra[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GemmDesc<R> g;
    g.C = d.ws + (int64_t)d.n * d.nrhs;
    g.A = d.Ainv;
    g.B = d.ws;
    g.ldc = g.lda = g.ldb = d.n > 0 ? d.n : 1;
    g.M = d.n;
    g.N = d.n > 0 ? d.nrhs : 0;
    g.K = d.n;
    g.beta = 0;
    g.sign = 1;
    desc[blockIdx.y] = g;
  }
  if (e >= (int64_t)d.n * d.nrhs) return;
  const int i = (int)(e % d.n), c = (int)(e / d.n);
  d.ws[e] = d.z[d.ids[i] + (int64_t)c * d.ldz];
}
template <class R>
__global__ void k_root_scatter_rhs(const RootApply<R>* ra) {
  const RootApply<R> d = ra[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d.n * d.nrhs) return;
  const int i = (int)(e % d.n), c = (int)(e / d.n);
  d.z[d.ids[i] + (int64_t)c * d.ldz] = d.ws[(int64_t)d.n * d.nrhs + e];
}
template <class R>
void launch_root_apply(const RootApply<R>* ra, int nprob, int max_n, int max_nrhs, GemmDesc<R>* desc,
                       hipStream_t s) {
  if (nprob == 0 || max_n == 0) return;
  const int64_t tot = (int64_t)max_n * max_nrhs;
  const dim3 g((unsigned)((tot + 255) / 256), nprob);
  hipLaunchKernelGGL(k_root_gather_rhs<R>, g, dim3(256), 0, s, ra, desc);
  launch_gemm<R>(desc, nprob, max_n, max_nrhs, s);
  hipLaunchKernelGGL(k_root_scatter_rhs<R>, g, dim3(256), 0, s, ra);
}

// ---------------------------------------------------------------------------
// kernel block evaluation (the FP64 on-the-fly residual is in rss_residual.hip)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kernel_block(KParams kp, const double* P, const int* I,
                                                      int64_t ni, const int* J, int64_t nj,
                                                      cx<double>* out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ni * nj) return;
  const int64_t i = e % ni, j = e / ni;
  out[e] = entry(kp, P, I[i], J[j]);
}

void launch_kernel_block(const KParams& kp, const double* P, const int* I, int64_t ni, const int* J,
                         int64_t nj, cx<double>* out, hipStream_t s) {
  const int64_t tot = ni * nj;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_kernel_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, kp, P, I,
                     ni, J, nj, out);
}

// ---------------------------------------------------------------------------
// refinement helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colnorms(const cx<double>* V, int64_t n, double* out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += abs2d(V[i + (int64_t)c * n]);
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[c] = sqrt(s);
}
void launch_colnorms(const cx<double>* V, int64_t n, int nrhs, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colnorms, dim3(nrhs), dim3(256), 0, s, V, n, out);
}

__global__ void k_scale_to_c64(const cx<double>* V, int64_t n, int nrhs, const double* norms,
                               cx<float>* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const double nr = norms[e / n];
  const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
  out[e] = cx<float>{(float)(V[e].x * sc), (float)(V[e].y * sc)};
}
void launch_scale_to_c64(const cx<double>* V, int64_t n, int nrhs, const double* norms,
                         cx<float>* out, hipStream_t s) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(k_scale_to_c64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, n,
                     nrhs, norms, out);
}

__global__ void k_axpy_from_c64(const cx<float>* d, int64_t n, int nrhs, const double* norms,
                                cx<double>* x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const double nr = norms ? norms[e / n] : 1.0;
  x[e].x += nr * (double)d[e].x;
  x[e].y += nr * (double)d[e].y;
}
void launch_axpy_from_c64(const cx<float>* d, int64_t n, int nrhs, const double* norms,
                          cx<double>* x, hipStream_t s) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(k_axpy_from_c64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, d, n,
                     nrhs, norms, x);
}

__global__ void k_cast_c64(const cx<double>* V, int64_t tot, cx<float>* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  out[e] = cx<float>{(float)V[e].x, (float)V[e].y};
}
void launch_cast_c64(const cx<double>* V, int64_t n, int nrhs, cx<float>* out, hipStream_t s) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(k_cast_c64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, tot, out);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

__global__ void k_add_c128(cx<double>* x, const cx<double>* d, int64_t tot) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < tot) x[e] = x[e] + d[e];
}
void launch_add_c128(cx<double>* x, const cx<double>* d, int64_t tot, hipStream_t s) {
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_add_c128, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, d, tot);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
#define RSS_INST(R)                                                                                \
  template void launch_leaf_assemble<R>(const Prob<R>*, int, int, int, hipStream_t);                    \
  template void launch_build_C<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t);              \
  template void launch_cpqr<R>(const Prob<R>*, const Phase<R>&, int, int, hipStream_t);            \
  template void launch_sparsify<R>(const Prob<R>*, const Phase<R>&, int, bool, hipStream_t);             \
  template void launch_inverse<R>(const Prob<R>*, const Phase<R>&, int*, int, hipStream_t);        \
  template void launch_plan_y<R>(const Prob<R>*, const Phase<R>&, GemmDesc<R>*, hipStream_t);      \
  template void launch_compact<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t);                   \
  template void launch_gemm<R>(const GemmDesc<R>*, int, int, int, hipStream_t);                    \
  template void launch_schur<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t);                \
  template void launch_assemble_pairs<R>(const PairDesc*, int, const ListEntry*, int, int,         \
                                         const Prob<R>*, hipStream_t);                             \
  template void launch_root_inverse<R>(const RootDesc<R>*, int, int, GemmDesc<R>*, int*, hipStream_t);           \
  template void launch_solve_fwd<R>(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, \
                                    cx<R>*, hipStream_t);                                          \
  template void launch_solve_bwd<R>(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, \
                                    cx<R>*, hipStream_t);                                          \
  template size_t solve_work_elems<R>(int, int, int, int);                                           \
  template void launch_root_apply<R>(const RootApply<R>*, int, int, int, GemmDesc<R>*, hipStream_t);  \
  template int cpqr_mg_groups<R>(int, int, int);                                                     \
  template int solve_group<R>(int, int, int);                                                        \
  template bool solve_fused_fits<R>(int, int, int);                                                  \
  template bool launch_cpqr_mg<R>(const Prob<R>*, const Phase<R>&, int, int, int, double*, double*,  \
                                  unsigned*, int*, unsigned, hipStream_t);

RSS_INST(double)
RSS_INST(float)

}  // namespace rss
