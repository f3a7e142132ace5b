// Internal interfaces of librss shared by the host driver (rss_host.cpp) and
// the device kernels (rss_kernels.hip).  Plain structs of device pointers and
// sizes, passed to kernels by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rss_device.h"

struct rss_ctx;  // a factorization handle (the C ABI's rss_handle)

namespace rss {

// One depth of the quadtree during factorization.
//  * box b (row-major id, nb x nb grid) owns the active global ids
//    idx[ioff[b] .. ioff[b] + cur[b]); capacity n0[b] = count at depth start.
//  * boff[25 b + s] is the offset into A of the dense block A[b, b2] for the
//    box b2 = b + (s % 5 - 2, s / 5 - 2) (Chebyshev distance <= 2), or -1 off
//    the grid.  The block is column-major with leading dimension n0[b] and
//    current size cur[b] x cur[b2].
template <class R>
struct Level {
  int d, nb;
  const int* n0;
  int* cur;
  int* idx;
  const int64_t* ioff;
  const int64_t* boff;
  cx<R>* A;
  double x0, y0, side;  // geometry of this depth's boxes (side = box side)
};

constexpr double TIE = 1e-8;  // pivot tie window of the interpolative decomposition

// box at offset (dx, dy) from b, or -1 off the grid
template <class R>
__device__ __forceinline__ int box_at(const Level<R>& L, int b, int dx, int dy) {
  const int bx = b % L.nb + dx, by = b / L.nb + dy;
  if (bx < 0 || by < 0 || bx >= L.nb || by >= L.nb) return -1;
  return by * L.nb + bx;
}

// the stored block A[b, b2] (b2 within distance 2 of b)
template <class R>
__device__ __forceinline__ cx<R>* block_ptr(const Level<R>& L, int b, int b2) {
  const int dx = b2 % L.nb - b % L.nb, dy = b2 / L.nb - b / L.nb;
  return L.A + L.boff[(int64_t)b * 25 + slot_of(dx, dy)];
}

// Factor records of the boxes of one depth (offsets are worst-case slots):
//  T     k x r      (ld k)         interpolation matrix, rows S, cols R ascending
//  Xi    r x r      (ld r)         X_RR^{-1}
//  XSNR  (k+nN) x r (ld k+nN)      [X_SR; X_NR]
//  Y     r x (k+nN) (ld r)         X_RR^{-1} [X_RS X_RN]
//  gS, gR, gN                      global ids of S, R and the neighbours' active sets
template <class R>
struct Records {
  int* k;
  int* r;
  int* nN;
  const int64_t* oT;
  const int64_t* oXi;
  const int64_t* oXSNR;
  const int64_t* oY;
  const int64_t* oS;
  const int64_t* oR;
  const int64_t* oN;
  cx<R>* F;
  int* G;
};

// One problem at one depth of a (possibly batched) factorization.
template <class R>
struct Prob {
  Level<R> L;
  Records<R> rec;
  KParams kp;
  const double* P;  // device points (n x 2)
  double tol;
  int n_proxy;
  double proxy_radius;
};

// One problem in a (possibly batched) solve sweep at one depth.
template <class R>
struct SolveProb {
  Records<R> rec;
  cx<R>* z;      // right-hand sides, column-major
  int64_t ldz;   // = number of points
  int nrhs;
};

// One colour phase: the boxes (of one or several problems) eliminated
// concurrently, and per-slot workspace.
template <class R>
struct Phase {
  int nbox;
  const int* box;
  const int* prob;     // problem index of each slot
  const int64_t* oC;   // compression matrix C (m x n, ld m) in W
  const int64_t* oX;   // X_RR (r x r) in W
  const int64_t* oZ;   // [X_RS X_RN] (r x (k+nN), ld r) in W
  const int64_t* oI;   // 3 n0 ints in Wi: Sloc, Rloc, perm
  int* mrow;           // rows of C per slot
  cx<R>* W;
  int* Wi;
  // r x r complex128 work for X_RR^{-1} when it does not fit in LDS
  const int64_t* oD;
  cx<double>* Wd;
  // solve sweeps: boxes of the phase share neighbours (four-colour
  // schedule), so the forward sweep's neighbour updates are atomic adds
  int atomic_nbr = 0;
};

// Workspace of the interpolative decomposition through the Gram matrix of one
// colour phase (FP64 arrays; every box's n is its active count n0[b]).
//  part : per slot, `chunks` partial Gram matrices, each hi (n x n) then lo
//  G    : per slot, the summed Gram matrix, hi then lo (aliases part when
//         chunks == 1)
//  Rw   : per slot, 2 (n x n): the rows of the pivoted Cholesky factor (high
//         parts, then T in their place), then their low parts
struct GramWs {
  double* part;
  const int64_t* oP;
  double* G;
  const int64_t* oG;
  double* Rw;
  const int64_t* oR;
  int chunks;      // row chunks per slot
  int chunk_rows;  // rows of Y (complex) per chunk
};

template <class R>
struct GemmDesc {
  cx<R>* C;
  const cx<R>* A;
  const cx<R>* B;
  int ldc, lda, ldb;
  int M, N, K;
  int beta;   // 0: C = sign A B; 1: C += sign A B
  int sign;   // +1 or -1
};

// Assembly of a dense block from the blocks of the depth below (Sec. 2.5,
// Fig. f:merge): rows/cols are lists of (child box, local position, global id).
struct PairDesc {
  void* dst;    // destination block (complex<R>, column-major, leading dimension ld)
  void* dstT;   // when not null, the transposed block too (leading dimension ldT):
                // a pair whose entries are all evaluated afresh (symmetric bit for bit)
  int ld, ldT;
  int nr, nc;
  int prob;     // problem index (child level, kernel, points)
  int have_child;
  int64_t roff, coff;  // into the entry list
};

// dense root of one problem: in-place Gauss-Jordan over A / tmp
template <class R>
struct RootDesc {
  cx<R>* A;        // n x n, inverted in place (before the final column interchanges)
  cx<R>* tmp;      // n x n: the inverse
  cx<R>* W;        // root_work_elems(n) entries: panel copy, panel rows, one column
  GemmDesc<R>* gd; // this problem's update product of the current panel
  int* perm;       // 2 n ints
  int n;
};
struct ListEntry {
  int box, local, gid;
};

// error flags written by kernels
enum { ERRF_SINGULAR = 1, ERRF_TIMEOUT = 2 };

// ---------------------------------------------------------------------------
// launchers (rss_kernels.hip); all enqueue on `s`
// ---------------------------------------------------------------------------
template <class R>
void launch_leaf_assemble(const Prob<R>* probs, int nprob, int max_boxes, int nmax, hipStream_t s);
template <class R>
void launch_build_C(const Prob<R>* probs, const Phase<R>& ph, int chunks, hipStream_t s);
template <class R>
void launch_cpqr(const Prob<R>* probs, const Phase<R>& ph, int nmax, int mmax, hipStream_t s);
// multi-workgroup ID for phases with few boxes: groups per box (1 = use launch_cpqr)
template <class R>
int cpqr_mg_groups(int nbox, int nmax, int mmax);
// right-hand sides per solve workgroup for the given largest skeleton and
// redundant counts of a level (0: the level's panels do not fit in LDS)
template <class R>
int solve_group(int kmax, int rmax, int nrhs);
// spin_limit bounds each per-box barrier wait (a timeout sets ERRF_TIMEOUT)
template <class R>
bool launch_cpqr_mg(const Prob<R>* probs, const Phase<R>& ph, int nmax, int mmax, int G,
                    double* pnorm, double* pdot, unsigned* bars, int* err, unsigned spin_limit, hipStream_t s);
// Interpolative decomposition through a double-double Gram matrix (boxes of
// at most GRAM_NMAX points): partial Gram matrices of row chunks, their sum,
// and the pivoted Cholesky factorization with T = R11^{-1} R12.
constexpr int GRAM_NMAX = 192;
// 4 x 4 tiles of the upper triangle of an n x n Gram matrix, in workgroups of 192 or 256
int gram_tile_groups(int nmax);
template <class R>
void launch_gram(const Prob<R>* probs, const Phase<R>& ph, const GramWs& gw, int nmax, hipStream_t s);
template <class R>
void launch_chol(const Prob<R>* probs, const Phase<R>& ph, const GramWs& gw, int nmax, hipStream_t s);
template <class R>
// treal: every T of the phase is real (IDs through the Gram matrix)
void launch_sparsify(const Prob<R>* probs, const Phase<R>& ph, int nmax, bool treal, hipStream_t s);
// LDS the sparsification needs at least (its S and R index lists) and the
// most it takes per workgroup
constexpr size_t SPARSIFY_LDS_CAP = (size_t)150 * 1024;
inline size_t sparsify_min_lds(int nmax) { return ((size_t)2 * nmax * sizeof(int) + 15) & ~(size_t)15; }
template <class R>
void launch_inverse(const Prob<R>* probs, const Phase<R>& ph, int* errflag, int nmax,
                    hipStream_t s);
template <class R>
void launch_plan_y(const Prob<R>* probs, const Phase<R>& ph, GemmDesc<R>* desc, hipStream_t s);
template <class R>
void launch_compact(const Prob<R>* probs, const Phase<R>& ph, int colours, hipStream_t s);
template <class R>
void launch_gemm(const GemmDesc<R>* desc, int ndesc, int max_m, int max_n, hipStream_t s);
// Schur update of every box of the phase as one (k + |N|)^2 product per box,
// scattered into the stencil blocks (qmax: bound on k + |N|)
template <class R>
void launch_schur(const Prob<R>* probs, const Phase<R>& ph, int qmax, hipStream_t s);
template <class R>
void launch_assemble_pairs(const PairDesc* pd, int npairs, const ListEntry* lists, int max_r,
                           int max_c, const Prob<R>* child, hipStream_t s);
template <class R>
void launch_root_inverse(const RootDesc<R>* rd, int nprob, int nmax, GemmDesc<R>* gd, int* errflag,
                         hipStream_t s);
// workspace entries of RootDesc::W for a root of size n
size_t root_work_elems(int n);
// Tile of the solve sweeps of one colour phase: ncg right-hand sides per
// workgroup (1 .. solve_group) and S workgroups per box for the two wide
// products (slices of their summation; 1 .. SOLVE_SMAX); fused: each sweep
// step in one launch, one workgroup per box (the arithmetic of S = 1).
struct SolveTile {
  int ncg, S;
  bool fused;
};
// whether the fused tile's LDS fits for a level
template <class R>
bool solve_fused_fits(int kmax, int rmax, int ncg);
constexpr int SOLVE_SMAX = 64;
// the default slice count: enough workgroups for the chip when a colour holds few boxes
int solve_slices(int nbox, int qmax);
// solve sweeps of one colour phase; W: scratch of solve_work_elems entries
// (qmax: largest k + |N| of the phase's level)
template <class R>
void launch_solve_fwd(const SolveProb<R>* sp, const Phase<R>& ph, int nrhs, int kmax, int rmax,
                      int qmax, SolveTile tile, cx<R>* W, hipStream_t s);
template <class R>
void launch_solve_bwd(const SolveProb<R>* sp, const Phase<R>& ph, int nrhs, int kmax, int rmax,
                      int qmax, SolveTile tile, cx<R>* W, hipStream_t s);
template <class R>
size_t solve_work_elems(int nbox, int rmax, int S, int nrhs);
// batched root apply: z[ids] <- Ainv z[ids] per problem (ws: 2 n nrhs entries per problem)
template <class R>
struct RootApply {
  const cx<R>* Ainv;
  const int* ids;
  int n;
  cx<R>* z;
  int64_t ldz;
  int nrhs;
  cx<R>* ws;
};
template <class R>
void launch_root_apply(const RootApply<R>* ra, int nprob, int max_n, int max_nrhs, GemmDesc<R>* desc,
                       hipStream_t s);

void launch_kernel_block(const KParams& kp, const double* P, const int* I, int64_t ni,
                         const int* J, int64_t nj, cx<double>* out, hipStream_t s);
// r = b - A x for several problems (FP64, on the fly)
struct ResDesc {
  KParams kp;
  const double* P;     // points, n x 2
  int64_t n;
  const cx<double>* X;  // n x nrhs, column-major (ld n), likewise B and R
  const cx<double>* B;
  cx<double>* R;
  cx<double>* part;     // S x 16 x n partial sums when S > 1
  const int* tperm;     // target order (spatially compact runs of 64), or null
  int nrhs;
  int S;                // source slices
};
struct ResBlock {
  int prob, tb, sp;     // problem, block of 256 targets, source slice
};
// source slices for a launch with this many 256-target blocks in total
int residual_slices(int64_t target_blocks);
// the allocation-free residual's scratch: device address of the current
// device's copy (nullptr if it cannot be obtained), RES_STATIC_BYTES long
constexpr size_t RES_STATIC_BYTES = (size_t)64 << 20;
constexpr int RES_STATIC_MAXDEV = 64;
void* residual_static_scratch();
// blk: every (problem, target block, slice); sum_blk: slice 0 of the target
// blocks of problems with S > 1
void launch_residual(const ResDesc* d, const ResBlock* blk, int nblk, const ResBlock* sum_blk,
                     int nsum, int max_nrhs, hipStream_t s);
// refinement helpers
void launch_colnorms(const cx<double>* V, int64_t n, int nrhs, double* out, hipStream_t s);
void launch_scale_to_c64(const cx<double>* V, int64_t n, int nrhs, const double* norms,
                         cx<float>* out, hipStream_t s);
void launch_axpy_from_c64(const cx<float>* d, int64_t n, int nrhs, const double* norms,
                          cx<double>* x, hipStream_t s);
void launch_cast_c64(const cx<double>* V, int64_t n, int nrhs, cx<float>* out, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_add_c128(cx<double>* x, const cx<double>* d, int64_t tot, hipStream_t s);

// Product with A on a uniform n x n grid of cell centres (x0 + (ix + 1/2) h,
// y0 + (iy + 1/2) h), user index iy n + ix, by FFT of an M x M circulant
// embedding of the Toeplitz part (M the power of two >= 2n - 1)
struct GridDesc {
  int n, M, logm;
  double x0, y0, h;
  KParams kp;
  const cx<double>* ghat;  // M x M, row-major [ky][kx]: FFT2 of the generator
  const cx<double>* tw;    // M / 2 twiddles exp(-2 pi i k / M)
  const double* scale;     // n^2 point scales
  const cx<double>* diag;  // n^2 diagonal entries
};
// generator transform (into C, which becomes ghat), point scales and diagonal
void launch_grid_setup(const GridDesc& g, cx<double>* C, double* scale, cx<double>* diag, hipStream_t s);
// Y = A X (mode 0) or Y = B - A X (mode 1), X, B, Y: n^2 x nrhs (ld), T: nrhs n M work
void launch_grid_apply(const GridDesc& g, const cx<double>* X, const cx<double>* B, cx<double>* Y, int64_t ld,
                       int nrhs, cx<double>* T, int mode, hipStream_t s);
// Krylov vector kernels: per-column conj(x).y (part: 64 nrhs entries of work),
// Y = a X + b Y with per-column a, b (null = 1), Y -= sum_j h_j V_j
void launch_cdot(const cx<double>* X, const cx<double>* Y, int64_t N, int nrhs, cx<double>* part,
                 cx<double>* out, hipStream_t s);
void launch_caxpby(const cx<double>* X, cx<double>* Y, int64_t N, int nrhs, const cx<double>* a,
                   const cx<double>* b, hipStream_t s);
void launch_lincomb_sub(const cx<double>* V, int64_t vstride, int k, const cx<double>* h, cx<double>* Y,
                        int64_t N, int nrhs, hipStream_t s);
constexpr int KRYLOV_DOT_BLOCKS = 64;

// refined solves a step at a time (the solve server's continuous batching):
// begin copies the right-hand sides; one step of several jobs (one precision)
// runs one batched application and one residual for all; finish writes the
// best iterate back, fills relres / iterations and frees the job
int refine_begin(::rss_ctx* h, void* B, int nrhs, void** job);
int refine_step(void* const* jobs, int n);
bool refine_done(const void* job);
int refine_finish(void* job, double* relres, int* iters);
void refine_free(void* job);

// set on the solve server's worker threads: batches of several handles there
// reuse tuned solve tiles but do not tune (see rss_set_autotune)
extern thread_local bool g_server_thread;

}  // namespace rss
