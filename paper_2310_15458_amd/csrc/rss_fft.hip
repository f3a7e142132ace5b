// Products with A for points on a uniform grid of cell centres, and the
// vector kernels of the Krylov iterations.
//
// On the grid x = (x0 + (ix + 1/2) h, y0 + (iy + 1/2) h), user index iy n + ix,
// the off-diagonal part of A is s_i g(ix - jx, iy - jy) s_j with
// g(dx, dy) = w K(h |(dx, dy)|): a block-Toeplitz matrix with Toeplitz blocks
// (Sec. 5 uses this structure for its products with A).  It is applied by
// FFT of an M x M circulant embedding, M the power of two >= 2n - 1:
//   A x = s * IFFT2(ghat * FFT2(pad(s * x))) + diag(A) * x,
// ghat = FFT2 of the generator placed at (dy mod M, dx mod M), 0 at the origin.
// The FFTs are radix-2 decimation in time in LDS, FP64, with a table of
// twiddles exp(-2 pi i k / M): one workgroup per row (rows of x, n of them;
// the other M - n rows of the padded array are zero), then one workgroup per
// group of columns (forward FFT, product with ghat, inverse FFT, only the
// n rows that the result needs written back), then the inverse row FFTs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rss_internal.h"

namespace rss {

__device__ __forceinline__ int bitrev(int i, int logm) {
  return (int)(__brev((unsigned)i) >> (32 - logm));
}

// `cnt` independent FFTs of length M in LDS (sequence s at a + s M, input in
// bit-reversed order, output in natural order); inverse: conjugate twiddles,
// unnormalized.  All threads of the workgroup take part.
__device__ void fft_lds(cx<double>* a, int cnt, int M, int logm, const cx<double>* tw, bool inv) {
  const int half = M >> 1;
  for (int s = 1; s <= logm; ++s) {
    const int len = 1 << s, hl = len >> 1, tstep = M >> s;
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * half; e += blockDim.x) {
      const int q = e / half, j = e - q * half;
      const int g = j / hl, pos = j - g * hl;
      cx<double>* b = a + (int64_t)q * M;
      const int i0 = g * len + pos, i1 = i0 + hl;
      cx<double> w = tw[pos * tstep];
      if (inv) w.y = -w.y;
      const cx<double> u = b[i0], v = b[i1];
      const cx<double> t{w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x};
      b[i0] = cx<double>{u.x + t.x, u.y + t.y};
      b[i1] = cx<double>{u.x - t.x, u.y - t.y};
    }
  }
  __syncthreads();
}

// generator of the circulant embedding, C[ky][kx] (row-major M x M)
__global__ __launch_bounds__(256) void k_grid_gen(GridDesc g, cx<double>* C) {
  const int M = g.M, n = g.n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * M) return;
  const int kx = (int)(e % M), ky = (int)(e / M);
  const int dx = kx < n ? kx : (kx > M - n ? kx - M : M);
  const int dy = ky < n ? ky : (ky > M - n ? ky - M : M);
  cx<double> v{0.0, 0.0};
  if (dx != M && dy != M && (dx != 0 || dy != 0)) {
    const cx<double> k = kernel_raw(g.kp, 0.0, 0.0, dx * g.h, dy * g.h);
    v = cx<double>{g.kp.weight * k.x, g.kp.weight * k.y};
  }
  C[e] = v;
}

// point scales and diagonal entries of the grid
__global__ __launch_bounds__(256) void k_grid_points(GridDesc g, double* scale, cx<double>* diag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)g.n * g.n) return;
  const int ix = (int)(i % g.n), iy = (int)(i / g.n);
  const double s = point_scale(g.kp, g.x0 + (ix + 0.5) * g.h, g.y0 + (iy + 0.5) * g.h);
  scale[i] = s;
  diag[i] = diag_entry(g.kp, s);
}

// forward FFT of the M rows of C in place (generator transform, rows pass)
__global__ __launch_bounds__(256) void k_fft_rows_inplace(GridDesc g, cx<double>* C) {
  extern __shared__ __align__(16) cx<double> fsm[];
  const int M = g.M;
  cx<double>* row = C + (int64_t)blockIdx.x * M;
  for (int x = threadIdx.x; x < M; x += 256) fsm[bitrev(x, g.logm)] = row[x];
  fft_lds(fsm, 1, M, g.logm, g.tw, false);
  for (int x = threadIdx.x; x < M; x += 256) row[x] = fsm[x];
}

// forward FFT of the columns of C in place (generator transform, columns pass)
__global__ __launch_bounds__(256) void k_fft_cols_inplace(GridDesc g, cx<double>* C, int cpw) {
  extern __shared__ __align__(16) cx<double> fsm[];
  const int M = g.M, kx0 = blockIdx.x * cpw;
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, y = e / cpw;
    fsm[(int64_t)j * M + bitrev(y, g.logm)] = C[(int64_t)y * M + kx0 + j];
  }
  fft_lds(fsm, cpw, M, g.logm, g.tw, false);
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, y = e / cpw;
    C[(int64_t)y * M + kx0 + j] = fsm[(int64_t)j * M + y];
  }
}

// rows of s * x, zero-padded to M, forward FFT -> T[c][iy][kx]
__global__ __launch_bounds__(256) void k_grid_rows_fwd(GridDesc g, const cx<double>* X, int64_t ldx,
                                                       cx<double>* T) {
  extern __shared__ __align__(16) cx<double> fsm[];
  const int M = g.M, n = g.n, iy = blockIdx.x, c = blockIdx.y;
  const cx<double>* xc = X + (int64_t)c * ldx + (int64_t)iy * n;
  const double* sc = g.scale + (int64_t)iy * n;
  for (int x = threadIdx.x; x < M; x += 256) {
    cx<double> v{0.0, 0.0};
    if (x < n) v = cx<double>{sc[x] * xc[x].x, sc[x] * xc[x].y};
    fsm[bitrev(x, g.logm)] = v;
  }
  fft_lds(fsm, 1, M, g.logm, g.tw, false);
  cx<double>* out = T + ((int64_t)c * n + iy) * M;
  for (int x = threadIdx.x; x < M; x += 256) out[x] = fsm[x];
}

// column groups: forward FFT over iy (rows >= n are zero), times ghat,
// inverse FFT, rows < n written back
__global__ __launch_bounds__(256) void k_grid_cols(GridDesc g, cx<double>* T, int cpw) {
  extern __shared__ __align__(16) cx<double> fsm[];
  const int M = g.M, n = g.n, kx0 = blockIdx.x * cpw, c = blockIdx.y;
  cx<double>* Tc = T + (int64_t)c * n * M;
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, y = e / cpw;
    fsm[(int64_t)j * M + bitrev(y, g.logm)] = y < n ? Tc[(int64_t)y * M + kx0 + j] : cx<double>{0.0, 0.0};
  }
  fft_lds(fsm, cpw, M, g.logm, g.tw, false);
  // product with ghat (each thread its own elements), then the bit-reversal
  // permutation in place for the inverse transform
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, ky = e / cpw;
    const cx<double> a = fsm[(int64_t)j * M + ky], b = g.ghat[(int64_t)ky * M + kx0 + j];
    fsm[(int64_t)j * M + ky] = cx<double>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, y = e / cpw, r = bitrev(y, g.logm);
    if (y < r) {
      cx<double>* col = fsm + (int64_t)j * M;
      const cx<double> t = col[y];
      col[y] = col[r];
      col[r] = t;
    }
  }
  fft_lds(fsm, cpw, M, g.logm, g.tw, true);
  for (int e = threadIdx.x; e < cpw * M; e += 256) {
    const int j = e % cpw, y = e / cpw;
    if (y < n) Tc[(int64_t)y * M + kx0 + j] = fsm[(int64_t)j * M + y];
  }
}

// inverse row FFTs; Y = s * z / M^2 + diag * X (mode 0) or R = B - that (mode 1)
__global__ __launch_bounds__(256) void k_grid_rows_inv(GridDesc g, const cx<double>* T, const cx<double>* X,
                                                       const cx<double>* B, cx<double>* Y, int64_t ld,
                                                       int mode) {
  extern __shared__ __align__(16) cx<double> fsm[];
  const int M = g.M, n = g.n, iy = blockIdx.x, c = blockIdx.y;
  const cx<double>* row = T + ((int64_t)c * n + iy) * M;
  for (int x = threadIdx.x; x < M; x += 256) fsm[bitrev(x, g.logm)] = row[x];
  fft_lds(fsm, 1, M, g.logm, g.tw, true);
  const double nrm = 1.0 / ((double)M * M);
  for (int x = threadIdx.x; x < n; x += 256) {
    const int64_t i = (int64_t)iy * n + x, e = (int64_t)c * ld + i;
    const double s = g.scale[i] * nrm;
    const cx<double> d = g.diag[i], xv = X[e];
    cx<double> v{s * fsm[x].x + d.x * xv.x - d.y * xv.y, s * fsm[x].y + d.x * xv.y + d.y * xv.x};
    if (mode == 1) v = cx<double>{B[e].x - v.x, B[e].y - v.y};
    Y[e] = v;
  }
}

// columns per workgroup: 64 KiB of LDS, at most all M columns
int grid_cols_per_wg(int M) { return std::min(M, std::max(1, 4096 / M)); }

void launch_grid_setup(const GridDesc& g, cx<double>* C, double* scale, cx<double>* diag, hipStream_t s) {
  const int64_t mm = (int64_t)g.M * g.M, nn = (int64_t)g.n * g.n;
  hipLaunchKernelGGL(k_grid_gen, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, g, C);
  hipLaunchKernelGGL(k_grid_points, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, g, scale, diag);
  const size_t row_lds = (size_t)g.M * sizeof(cx<double>);
  hipLaunchKernelGGL(k_fft_rows_inplace, dim3(g.M), dim3(256), row_lds, s, g, C);
  const int cpw = grid_cols_per_wg(g.M);
  hipLaunchKernelGGL(k_fft_cols_inplace, dim3(g.M / cpw), dim3(256), row_lds * cpw, s, g, C, cpw);
}

void launch_grid_apply(const GridDesc& g, const cx<double>* X, const cx<double>* B, cx<double>* Y, int64_t ld,
                       int nrhs, cx<double>* T, int mode, hipStream_t s) {
  const size_t row_lds = (size_t)g.M * sizeof(cx<double>);
  const int cpw = grid_cols_per_wg(g.M);
  hipLaunchKernelGGL(k_grid_rows_fwd, dim3(g.n, nrhs), dim3(256), row_lds, s, g, X, ld, T);
  hipLaunchKernelGGL(k_grid_cols, dim3(g.M / cpw, nrhs), dim3(256), row_lds * cpw, s, g, T, cpw);
  hipLaunchKernelGGL(k_grid_rows_inv, dim3(g.n, nrhs), dim3(256), row_lds, s, g, T, X, B, Y, ld, mode);
}

// ---------------------------------------------------------------------------
// vector kernels of the Krylov iterations; every vector is N x nrhs,
// column-major (leading dimension N); per-column scalars in device arrays
// ---------------------------------------------------------------------------
constexpr int DOT_BLOCKS = KRYLOV_DOT_BLOCKS;

// partial sums of conj(x_c) . y_c: block b of column c sums rows b, b + 64*256, ...
__global__ __launch_bounds__(256) void k_cdot_part(const cx<double>* X, const cx<double>* Y, int64_t N,
                                                   cx<double>* part) {
  __shared__ double sr[256], si[256];
  const int b = blockIdx.x, c = blockIdx.y;
  const cx<double>* x = X + (int64_t)c * N;
  const cx<double>* y = Y + (int64_t)c * N;
  double ar = 0.0, ai = 0.0;
  for (int64_t i = (int64_t)b * 256 + threadIdx.x; i < N; i += (int64_t)DOT_BLOCKS * 256) {
    ar += x[i].x * y[i].x + x[i].y * y[i].y;
    ai += x[i].x * y[i].y - x[i].y * y[i].x;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)c * DOT_BLOCKS + b] = cx<double>{sr[0], si[0]};
}

// the blocks' partial sums in order (deterministic)
__global__ void k_cdot_sum(const cx<double>* part, int nrhs, cx<double>* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  cx<double> s{0.0, 0.0};
  for (int b = 0; b < DOT_BLOCKS; ++b) s = s + part[(int64_t)c * DOT_BLOCKS + b];
  out[c] = s;
}

void launch_cdot(const cx<double>* X, const cx<double>* Y, int64_t N, int nrhs, cx<double>* part,
                 cx<double>* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cdot_part, dim3(DOT_BLOCKS, nrhs), dim3(256), 0, s, X, Y, N, part);
  hipLaunchKernelGGL(k_cdot_sum, dim3((nrhs + 63) / 64), dim3(64), 0, s, part, nrhs, out);
}

// Y_c = a_c X_c + b_c Y_c (a, b per column; either may be null for 1)
__global__ void k_caxpby(const cx<double>* X, cx<double>* Y, int64_t N, const cx<double>* a,
                         const cx<double>* b) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const cx<double> ac = a ? a[c] : cx<double>{1.0, 0.0};
  const cx<double> bc = b ? b[c] : cx<double>{1.0, 0.0};
  const cx<double> x = X[(int64_t)c * N + i], y = Y[(int64_t)c * N + i];
  Y[(int64_t)c * N + i] = cx<double>{ac.x * x.x - ac.y * x.y + bc.x * y.x - bc.y * y.y,
                                     ac.x * x.y + ac.y * x.x + bc.x * y.y + bc.y * y.x};
}

void launch_caxpby(const cx<double>* X, cx<double>* Y, int64_t N, int nrhs, const cx<double>* a,
                   const cx<double>* b, hipStream_t s) {
  hipLaunchKernelGGL(k_caxpby, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, X, Y, N, a, b);
}

// Y_c -= sum_{j < k} h[j * nrhs + c] V_j,c  (the Gram-Schmidt update of GMRES)
__global__ void k_lincomb_sub(const cx<double>* V, int64_t vstride, int k, const cx<double>* h, cx<double>* Y,
                              int64_t N, int nrhs) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  cx<double> y = Y[(int64_t)c * N + i];
  for (int j = 0; j < k; ++j) {
    const cx<double> hj = h[(int64_t)j * nrhs + c], v = V[(int64_t)j * vstride + (int64_t)c * N + i];
    y = cx<double>{y.x - (hj.x * v.x - hj.y * v.y), y.y - (hj.x * v.y + hj.y * v.x)};
  }
  Y[(int64_t)c * N + i] = y;
}

void launch_lincomb_sub(const cx<double>* V, int64_t vstride, int k, const cx<double>* h, cx<double>* Y,
                        int64_t N, int nrhs, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_lincomb_sub, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, V, vstride, k, h,
                     Y, N, nrhs);
}

}  // namespace rss
