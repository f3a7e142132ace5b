/*
 * rss.h -- C ABI of librss: strong recursive skeletonization (RS-S) on one
 * AMD MI355X (gfx950).
 *
 * The library factors the dense kernel matrix of a planar integral equation,
 *   A x = b,  A_ij = w K(|x_i - x_j|) (i != j),  A_ii = d            (Sec. 1, eqs. e:axb, e:aij)
 * into the compressed inverse of Sec. 2 (Alg. a:fact with the multilevel
 * recursion of Sec. 2.5) and applies it to right-hand sides (Sec. 2.6).
 * Kernels: 2-D Laplace K = -log(r)/(2 pi) (eq. e:kernel_laplace) and 2-D
 * Helmholtz K = (i/4) H0^(1)(kappa r) (eq. e:kernel_helmholtz), plus the
 * exactly low-rank test kernel (1 + x.y)^q.
 *
 * Conventions for every entry point:
 *  - Return value: RSS_OK (0) or a negative rss_status.  rss_last_error()
 *    returns a message for the last failure on the calling thread.
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - Device pointers are HIP device memory of the current device.
 *  - Dense matrices are complex, column-major, interleaved (re, im).
 *  - Work is ordered on the handle's stream (rss_options.stream, or a stream
 *    the library owns); every call returns after its work has completed.
 *  - A handle must not be used by two threads at once.
 */
#ifndef RSS_H
#define RSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSS_OK = 0,
  RSS_EINVAL = -1,        /* bad argument: null pointer, n < 1, tol <= 0, leaf < 1,
                             nrhs < 1, non-finite or coincident points (two points with
                             equal x and y), kappa <= 0 for Helmholtz */
  RSS_ENOMEM = -2,        /* device allocation failed or the memory budget is exceeded */
  RSS_EUNSUPPORTED = -3,  /* e.g. a tree deeper than 15 levels or more than 2^31-1 points */
  RSS_ESINGULAR = -4,     /* an exactly zero pivot in a redundant-block or root LU */
  RSS_ENOCONV = -5,       /* refinement stopped at max_refine above refine_tol;
                             the output holds the best iterate */
  RSS_EHIP = -6           /* a HIP runtime call failed */
} rss_status;

typedef enum {
  RSS_LAPLACE2D = 0,      /* K = -log(r) / (2 pi)            (eq. e:kernel_laplace) */
  RSS_HELMHOLTZ2D = 1,    /* K = (i/4) H0^(1)(kappa r)        (eq. e:kernel_helmholtz) */
  RSS_DEGENERATE = 2      /* K = (1 + x.y)^q, exactly low rank (test kernel) */
} rss_kernel_kind;

typedef struct {
  rss_kernel_kind kind;
  double kappa;           /* Helmholtz wavenumber (> 0) */
  double weight;          /* w: off-diagonal entries are w s_i s_j K(x_i, x_j) (quadrature weight h^2) */
  double diag;            /* d: diagonal entries A_ii = d (+ the cell term below) */
  int q;                  /* degree of the degenerate kernel */
  /* The paper's discretizations (Sec. 5); all zero: s = 1, A_ii = d.
   *   cell_diag != 0: A_ii = d + (w / h^2) s_i^2 c(h) with c(h) the integral of K
   *     over an h x h cell centred at the point (eqs. e:a1i, e:b2), computed by the
   *     library (Laplace and Helmholtz kernels; h > 0 required).
   *   bump_a > 0: scattering potential b(x) = exp(-bump_a |x - bump_c|^2) and point
   *     scale s_i = sqrt(b(x_i)) (the symmetrized Lippmann-Schwinger form, eq. e:b1).
   * First-kind Laplace (eqs. e:a1, e:a1i): w = h^2, d = 0, cell_diag.  LS Helmholtz
   * (eqs. e:b1, e:b2): w = h^2 kappa^2, d = 1, cell_diag, bump_a = 32, bump_c = (1/2, 1/2). */
  int cell_diag;
  double h;
  double bump_a;
  double bump_c[2];
} rss_kernel;

typedef enum {
  RSS_FP64 = 0,           /* factor and solve in complex128 */
  RSS_FP32_REFINE = 1     /* factor and solve in complex64; rss_solve refines in FP64 */
} rss_precision;

/* Zero-initialised means "all defaults". */
typedef struct {
  int n_proxy;            /* proxy points per circle; 0 -> 64 (Laplace/degenerate), 128 (Helmholtz) */
  double proxy_radius;    /* proxy circle radius in box-side units; 0 -> 1.25 (Sec. 2.3) */
  rss_precision precision;
  double refine_tol;      /* stop refining when max_j ||A x_j - b_j|| / ||b_j|| <= refine_tol; 0 -> 1e-10 */
  int max_refine;         /* refinement steps after the first solve; 0 -> 10; < 0 -> never refine
                             (RSS_FP64 never refines unless max_refine > 0) */
  double root[3];         /* x0, y0, side of the root square; side <= 0 -> [0,1]^2 if every
                             point lies in it, else the bounding square */
  void* stream;           /* hipStream_t for all work; NULL -> a stream owned by the handle */
  int profile;            /* nonzero: time every kernel class with HIP events on the stream
                             (rss_stats.t_class_ms); adds a little host overhead */
  int colours;            /* elimination schedule within a depth; 0 or 9: nine colours
                             (bx mod 3) + 3 (by mod 3), boxes of a colour 3 apart, the default;
                             4: four colours (bx mod 2) + 2 (by mod 2) (Sec. 3's coloured
                             variant: only neighbours differ): boxes of a colour are 2 apart,
                             every ID of a colour is taken before its first elimination, their
                             Schur updates meet additively (applied in four ordered passes, so
                             the factorization is deterministic) and the forward solve adds
                             their neighbour updates atomically (results not bitwise
                             reproducible).  Fewer, wider phases: 4 instead of 9 per depth.
                             All problems of one rss_factor_batch share the schedule. */
} rss_options;

/* kernel classes timed when rss_options.profile is set (index into t_class_ms) */
enum {
  RSS_K_ASSEMBLE = 0,     /* leaf blocks, transition and root assembly */
  RSS_K_BUILD_C = 1,      /* compression matrices (eqs. e:con, e:proxy) */
  RSS_K_ID = 2,           /* column-pivoted QR interpolative decomposition (Def. 1) */
  RSS_K_SPARSIFY = 3,     /* sparsification (eq. e:s) */
  RSS_K_INVERSE = 4,      /* redundant-block inverse (the LU of eq. e:step) */
  RSS_K_GEMM_Y = 5,       /* Y = X_RR^{-1} [X_RS X_RN] */
  RSS_K_COMPACT = 6,      /* dropping the redundant rows and columns */
  RSS_K_SCHUR = 7,        /* Schur-complement update (eq. e:step) */
  RSS_K_ROOT = 8,         /* dense root inverse */
  RSS_K_NCLASS = 12
};

typedef struct rss_ctx* rss_handle;

/*
 * rss_factor / rss_factor_ex -- build the RS-S factorization (Alg. a:fact).
 *   points : host, n x 2 float64, row-major (x_i = points[2i], y_i = points[2i+1]).
 *   n      : number of points (1 .. 2^31-1); row i of every right-hand side
 *            belongs to points[i].
 *   k      : kernel description (host, copied).
 *   tol    : ID tolerance eps of Def. 1 (> 0): a box keeps the fewest
 *            column-pivoted-QR pivots after which every trailing column norm
 *            is <= tol * |R_00| of its compression matrix.
 *   leaf   : maximum points per leaf box; the tree depth D is the smallest
 *            depth at which no box holds more than leaf points (Sec. 2.1).
 *   opt    : options (may be NULL in rss_factor_ex).
 *   out    : receives the handle; set to NULL on failure.
 * The handle owns all device memory of the factorization until rss_free.
 */
int rss_factor(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
               rss_handle* out);
int rss_factor_ex(const double* points, int64_t n, const rss_kernel* k, double tol, int leaf,
                  const rss_options* opt, rss_handle* out);

/*
 * rss_solve -- overwrite B with A^{-1} B applied through the factorization
 * (Sec. 2.6: upward pass, root solve, downward pass).
 *   B    : device, complex128, n x nrhs, column-major, leading dimension n.
 *   nrhs : number of columns (>= 1).
 * In RSS_FP32_REFINE form (and in RSS_FP64 form with max_refine > 0) the
 * result is refined: r = b - A x is evaluated in FP64 directly from the
 * kernel (O(n^2) per step) and x += F^{-1} r until refine_tol is met.
 * Returns RSS_ENOCONV (with the best iterate in B) if it is not met.
 */
int rss_solve(rss_handle h, void* B, int nrhs);

/*
 * rss_solve_batch -- rss_solve for several factorizations at once: every
 * application of the factored inverses is one batched sweep over all problems
 * that are still refining.  All handles must share precision and refinement
 * mode; work runs on the stream of hs[0].  B[p]: device complex128,
 * n_p x nrhs[p], column-major, overwritten.  Returns RSS_ENOCONV if any
 * problem missed its refine_tol (every B[p] holds the best iterate).
 */
int rss_solve_batch(int nh, rss_handle* hs, void* const* B, const int* nrhs);

/* rss_apply -- one application of the factored inverse, no refinement. */
int rss_apply(rss_handle h, void* B, int nrhs);

/*
 * rss_factor_batch -- factor nprob independent problems together: at every
 * height above the leaves, each colour phase is one set of launches over the
 * boxes of all problems that have that depth (Alg. a:fact applied to each
 * problem; the problems share no data).
 *   points[p], n[p], kernels[p] : as in rss_factor for problem p.
 *   tol, leaf, opt              : shared by all problems (opt->n_proxy = 0 picks
 *                                 the per-kernel default for each problem).
 *   out                         : nprob handles, each usable and freed on its own;
 *                                 all NULL on failure.
 * The handles share one stream (opt->stream, or one the library creates and
 * destroys with the last of them).
 */
int rss_factor_batch(int nprob, const double* const* points, const int64_t* n,
                     const rss_kernel* kernels, double tol, int leaf, const rss_options* opt,
                     rss_handle* out);

/*
 * rss_apply_batch -- one application of each factored inverse to its own
 * right-hand sides, all problems in one set of launches per (height, colour).
 *   hs[p]   : handles of one precision.  B[p] : device complex128, n_p x nrhs[p],
 *   column-major, overwritten.  Work runs on the stream of hs[0].
 */
int rss_apply_batch(int nh, rss_handle* hs, void* const* B, const int* nrhs);

/* rss_free -- release the handle and its device memory (NULL is a no-op). */
void rss_free(rss_handle h);

typedef struct {
  int64_t n;              /* number of points */
  int depth;              /* leaf depth D (root is depth 0) */
  int precision;          /* rss_precision of the factorization */
  int n_root;             /* size of the dense root block */
  int64_t boxes_compressed;
  int64_t rank_sum[16];   /* sum of skeleton counts k over the boxes of each depth */
  int64_t box_count[16];  /* non-empty boxes of each depth */
  int64_t redundant_sum[16];
  double flops_id;        /* ledger (real flops, a complex multiply-add counts 8) */
  double flops_lu;
  double flops_y;
  double flops_schur;
  double factor_bytes;    /* bytes of stored factor entries (what a solve streams) */
  double kernel_evals;    /* kernel evaluations during the factorization */
  double t_factor_ms;     /* wall time of the last rss_factor on the device stream */
  double t_solve_ms;      /* wall time of the last rss_solve */
  double last_relres;     /* max column relative residual of the last refined solve (-1: none) */
  int last_iters;         /* refinement steps taken by the last rss_solve */
  double device_bytes;    /* device memory held by the handle */
  double t_class_ms[12];  /* per kernel class, summed over launches (rss_options.profile) */
  int64_t n_class[12];    /* launches per kernel class */
  int id_retries;         /* 1 if the factorization was redone with the single-workgroup QR
                             after a multi-workgroup barrier timed out (boxes above 192 points) */
} rss_stats;

/* rss_info -- statistics of a factorization (host struct filled). */
int rss_info(rss_handle h, rss_stats* s);

/*
 * rss_skeletons -- the skeleton set chosen for every box of one depth.
 *   depth  : D .. 2 (compressed depths).
 *   counts : host, 4^depth int32, receives k per box (-1 for empty boxes).
 *   ids    : host, receives the skeleton point indices of every box in box-id
 *            order, each box's ascending; may be NULL to query the total.
 *   cap    : capacity of ids; total : receives the number of ids.
 */
int rss_skeletons(rss_handle h, int depth, int32_t* counts, int64_t* ids, int64_t cap,
                  int64_t* total);

/*
 * rss_kernel_block -- evaluate the kernel matrix block A[I, J] on the device
 * (entries as in rss_factor: w K off the diagonal, d where I[a] == J[b]).
 *   points : device, n x 2 float64 row-major.   I, J : device int32 index arrays.
 *   out    : device complex128, ni x nj column-major.
 *   stream : hipStream_t (NULL = default stream).
 */
int rss_kernel_block(const rss_kernel* k, const double* points, int64_t n, const int32_t* I,
                     int64_t ni, const int32_t* J, int64_t nj, void* out, void* stream);

/*
 * rss_residual -- R = B - A X in FP64, every entry of A evaluated from the
 * kernel on the fly (O(n^2 nrhs)); the refinement residual of rss_solve.
 *   points : device, n x 2 float64 row-major.  X, B, R : device complex128,
 *   n x nrhs column-major (ld n).  R may alias B.
 */
int rss_residual(const rss_kernel* k, const double* points, int64_t n, const void* X,
                 const void* B, void* R, int nrhs, void* stream);

/*
 * rss_residual_static -- rss_residual without any device allocation, for
 * callers that cannot allocate (code under stream capture, serving loops
 * with a fixed memory footprint, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results as rss_residual; its target order,
 * descriptors and source-slice partial sums live in a 64 MiB array that the
 * library holds on every device it runs on until the process ends.
 *   n : at most about 16 million points (the target order and one slice must
 *       fit; larger n returns RSS_EINVAL).  Fewer source slices than
 *       rss_residual chooses are used when their partial sums do not fit,
 *       which changes results at the rounding level only.
 * Calls on one device share that array: calls that overlap in time on the
 * same device (other threads, other streams) race and must not be made.
 * Returns after the work has completed on `stream`.
 */
int rss_residual_static(const rss_kernel* k, const double* points, int64_t n, const void* X,
                        const void* B, void* R, int nrhs, void* stream);

/* ------------------------------------------------------------------------- */
/* Products with A on a uniform grid, and factorization-preconditioned CG /  */
/* GMRES (Sec. 5, Tab. t:notations n_it).                                    */
/* ------------------------------------------------------------------------- */
typedef struct rss_gridop* rss_gridop_t;

/*
 * rss_gridop_create -- the product with A for the n x n grid of cell centres
 * x = (x0 + (ix + 1/2) h, y0 + (iy + 1/2) h), point index iy n + ix (Sec. 5:
 * A is block-Toeplitz with Toeplitz blocks there, applied by FFT of a
 * circulant embedding of side the power of two >= 2n - 1).
 *   k      : kernel and entry rule as in rss_factor (Laplace or Helmholtz).
 *   n      : 1 .. 2048.   stream : hipStream_t of the operator's own calls
 *            (NULL: one the operator creates).
 * Holds ~(2n)^2 complex128 of device memory plus a work array that grows to
 * nrhs n (2n) entries.  Not for concurrent use from several threads.
 */
int rss_gridop_create(const rss_kernel* k, int n, double x0, double y0, double h, void* stream,
                      rss_gridop_t* out);
/* rss_gridop_apply -- Y = A X; X, Y: device complex128, n^2 x nrhs column-major. */
int rss_gridop_apply(rss_gridop_t op, const void* X, void* Y, int nrhs);
/* rss_gridop_residual -- R = B - A X (R may alias B). */
int rss_gridop_residual(rss_gridop_t op, const void* X, const void* B, void* R, int nrhs);
/* rss_gridop_free -- release the operator (NULL is a no-op). */
void rss_gridop_free(rss_gridop_t op);

/*
 * rss_set_residual_op -- refined solves of this handle (rss_solve,
 * rss_solve_batch) take their residual r = b - A x from the grid operator
 * (FFT, FP64) instead of the on-the-fly O(n^2) sum.  op must describe the same
 * matrix (points in the operator's order, the same kernel) and outlive its use;
 * NULL restores the on-the-fly residual.  RSS_EINVAL if the sizes differ.
 */
int rss_set_residual_op(rss_handle h, rss_gridop_t op);

typedef struct {
  int iters;              /* iterations taken (the largest over the columns) */
  double relres;          /* max over columns of ||A x - b|| / ||b||, A by the grid operator */
  double t_ms;            /* wall time on the handle's stream */
} rss_krylov_stats;

/*
 * rss_krylov -- solve A x = b by a Krylov method preconditioned by the
 * factorization, as Sec. 5 does: method 0 conjugate gradients (for Hermitian
 * positive definite A, e.g. first-kind Laplace), method 1 GMRES without
 * restart (right preconditioning; e.g. Lippmann-Schwinger Helmholtz).
 * Products with A by the grid operator, the preconditioner F^{-1} applied in
 * the handle's precision.  B: device complex128, n x nrhs column-major, the
 * right-hand sides in, the solutions out; columns iterate together until each
 * reaches ||r|| <= tol ||b|| or maxit iterations.  st may be NULL.
 */
int rss_krylov(rss_handle h, rss_gridop_t A, void* B, int nrhs, int method, double tol, int maxit,
               rss_krylov_stats* st);

/*
 * rss_krylov_ex -- rss_krylov with restarts and an optional preconditioner:
 * restart m > 0 runs GMRES(m) (each cycle of at most m steps starts again
 * from the true residual b - A x; m = 0: no restart; ignored by CG); h may
 * be NULL for the unpreconditioned iteration (Tab. t:h2 counts GMRES(20)
 * iterations without a preconditioner), the work then runs on `stream` (a
 * hipStream_t; NULL: the grid operator's stream).  maxit bounds the total
 * number of iterations over all cycles.
 */
int rss_krylov_ex(rss_handle h, rss_gridop_t A, void* B, int nrhs, int method, double tol, int maxit,
                  int restart, void* stream, rss_krylov_stats* st);

/*
 * rss_set_stream -- move a handle's later work to another stream (hipStream_t;
 * NULL is not allowed).  The caller orders it after work already queued.
 */
int rss_set_stream(rss_handle h, void* stream);

/*
 * rss_set_graphs -- process-wide switch (default on) for the captured solve
 * sweeps of Sec. 2.6: with it on, an apply of a single handle (rss_apply,
 * rss_solve and each refinement step) replays a HIP
 * graph of all its launches, captured on the handle's first apply with that
 * nrhs and kept until rss_free (at most 4 per handle, the least recently used
 * dropped; their descriptors and workspace are device memory beyond
 * rss_stats.device_bytes); the vectors are reached through descriptor
 * tables in device memory that each call rewrites before the replay.  Off:
 * every apply launches its kernels directly (the same kernels, same results).
 * Batches of several handles, and every apply of the solve server, always
 * launch directly.  The capture runs in thread-local mode on the handle's
 * stream, but HIP still rejects some calls (frees among them) made by other
 * threads while it lasts: a program that calls the library from several
 * threads at once should switch graphs off (the server needs nothing: it
 * never captures).  enable: 0 or 1; returns the previous setting.
 */
int rss_set_graphs(int enable);

/*
 * rss_trim_cache -- return the current device's cached device memory to the
 * driver.  Freed factor records and workspaces stay with the library, per
 * size class, and serve later allocations (repeated and batched
 * factorizations then allocate nothing from the driver); the cache keeps at
 * most three quarters of the device's memory, and gives blocks back by itself
 * when one of the library's own allocations fails, but not when other code in
 * the process (torch's allocator, for one) runs short: such a caller trims
 * first.  A program that moves on to a different workload (other problem
 * sizes or counts) trims too: once the cache is full of the old workload's
 * blocks, frees past the cap go back with hipFree, which synchronizes the
 * device and, inside a factorization, stalls its launches.
 * Blocks in use by live handles or servers are not touched.  released (may be
 * NULL): the bytes returned.  RSS_OK, or RSS_EHIP if no device is current.
 */
int rss_trim_cache(int64_t* released);

/*
 * rss_set_autotune -- process-wide switch (default on) for the solve's tile
 * autotuner.  Each level of a solve (one tree height of one or more handles)
 * runs its sweeps with a tile: the right-hand sides per workgroup and the
 * workgroups per box of its two wide products.  With the switch on, the first
 * apply that meets a level shape not seen before (precision; largest group
 * width and box count, each rounded up to a power of two; largest skeleton
 * and redundant counts rounded up to 8; largest k + |N| rounded up to 32) times the candidate tiles on that apply's own shapes (on
 * vectors of zeros: the caller's data is untouched) and keeps the fastest for
 * the rest of the process; later applies of that shape, across handles and
 * servers, reuse it.  Off: untuned shapes use the default tile.  A tile that
 * splits a summation differently changes results at the rounding level only.
 * Inside the solve server, batches that merge several handles reuse what is
 * tuned and otherwise take the default tile (no tuning on request latency).
 * The candidates per level: 1, 1/2 or 1/4 of the widest group that fits the
 * LDS budget; half, the default or twice the default workgroups per box; and
 * the fused tile (each sweep step in one launch, one workgroup per box).
 * enable: 0 (off), 1 (on) or 2 (no timing: every level takes the fused tile
 * where its LDS fits, the default tile elsewhere; for tests and comparisons).
 * Returns the previous setting, or RSS_EINVAL for another value.
 */
int rss_set_autotune(int enable);

/*
 * Factor-side tuning (same switch, enable = 1 only): the ID's Gram kernel
 * splits each box's rows into chunks, one workgroup each; per bucket of
 * (precision, largest box in steps of 16 points, log2 of the boxes in the
 * launch, log2 of the rows of a box) the first phase of a factorization that
 * meets the bucket times the chunkings that aim at 512, 1024, 2048, 4096 and
 * 8192 workgroups on its own data and keeps the fastest for the process
 * (later phases and factorizations reuse it; the solve server's threads
 * never time).  Off: 2048.  The choice changes only the order in which
 * partial Gram matrices are summed (double-double, Def. 1's decisions are
 * taken on it).
 *
 * rss_factor_tuning -- copy up to cap entries of the table into out and set
 * *count to the number of entries; out may be NULL with cap 0.
 * rss_factor_tuning_clear -- empty the table (the next factorizations tune again).
 */
typedef struct {
  int precision_bytes;    /* 4: complex64 factors, 8: complex128 */
  int box_points_hi;      /* the bucket holds boxes of up to this many points */
  int boxes_log2;         /* ... launches of up to 2^boxes_log2 boxes */
  int rows_log2;          /* ... boxes of up to 2^rows_log2 rows */
  int target_workgroups;  /* the chosen target */
  int chunks;             /* the row chunks per box it gave */
  float us;               /* its measured time per launch */
} rss_tune_entry;
int rss_factor_tuning(rss_tune_entry* out, int cap, int* count);
int rss_factor_tuning_clear(void);

/* ------------------------------------------------------------------------- */
/* Solve server: factorizations stay resident in device memory; factor and   */
/* solve requests are served with continuous batching (a factor worker and a */
/* solve worker on separate streams, so factor and solve work overlap).      */
/* The solve worker advances every solve in flight by one step at a time --  */
/* one batched application of the factored inverses (Sec. 2.6) over all of   */
/* them, then one residual per solve -- admitting newly arrived solves at    */
/* every step boundary (up to max_batch in flight) and retiring each as soon */
/* as it has converged.                                                      */
/* ------------------------------------------------------------------------- */
typedef struct rss_server* rss_server_t;

typedef struct {
  double budget_bytes;    /* device memory of the server.  Three quarters are for resident
                             factorizations: new factor jobs wait for room, least-recently-used
                             unpinned ones are evicted (the size of a job is estimated from the
                             largest bytes per unknown seen so far; an empty server always
                             admits a job).  One quarter is for the working buffers of solves
                             in flight (about 72 bytes per unknown and right-hand side with
                             refinement in FP32, 64 in FP64): a solve waits until its buffers
                             fit (a solve alone is always admitted) */
  int precision;          /* rss_precision of every factorization */
  double tol;             /* ID tolerance (Def. 1) */
  int leaf;               /* points per leaf box */
  int n_proxy;            /* 0 -> per-kernel default */
  double refine_tol;      /* as rss_options */
  int max_refine;         /* as rss_options */
  int max_batch;          /* most solves in flight (one batched step); 0 -> 64 */
  int grid_residual;      /* nonzero: a factorization whose points form a uniform grid of cell
                             centres (rows of n x n cells, point index iy n + ix) refines with the
                             FFT grid product (rss_gridop_*) as its residual */
} rss_server_options;

typedef struct {
  int64_t req;            /* request id (for a factor request: the factorization id) */
  int kind;               /* 0 factor, 1 solve */
  int status;             /* rss_status of the request */
  double t_submit, t_start, t_end;  /* seconds since the server started */
  double relres;          /* refined solves: max column relative residual; else -1 */
  int iters;              /* refinement steps */
  int batch;              /* solves in flight in the step that completed it */
} rss_completion;

typedef struct {
  /* batches: batched steps run; batched_solves: sum over steps of the solves in flight;
     max_batch_seen: most solves in one step */
  int64_t factored, evictions, batches, batched_solves, max_batch_seen, resident, pending;
  double used_bytes, peak_bytes;   /* resident factorizations: now, and the most */
  double solved_unknowns; /* sum over completed solves of n * nrhs */
  double inflight_bytes, inflight_peak_bytes;  /* working buffers of solves in flight */
  int64_t refactors;      /* evicted factorizations factored again for a solve */
} rss_server_stats;

/* rss_server_create -- start the workers.  Returns RSS_EINVAL on bad options. */
int rss_server_create(const rss_server_options* o, rss_server_t* out);
/* rss_server_factor -- queue a factorization (points: host n x 2, copied); *id names it. */
int rss_server_factor(rss_server_t s, const double* points, int64_t n, const rss_kernel* k,
                      int64_t* id);
/* rss_server_solve -- queue a solve against factorization id, pinning it until the solve
 * completes.  A factorization that was evicted is factored again first (the server keeps
 * every problem's points and kernel on the host; that factor job reports no completion).
 * B: device complex128 n x nrhs column-major, overwritten with the solution; the caller
 * must not touch it before completion.  RSS_EINVAL for an unknown id or one whose
 * factorization failed. */
int rss_server_solve(rss_server_t s, int64_t id, void* B, int nrhs, int64_t* req);
/* rss_server_poll -- take up to cap completions, waiting up to wait_ms for the first. */
int rss_server_poll(rss_server_t s, rss_completion* out, int cap, int wait_ms, int* count);
/* rss_server_stats_get -- counters of the server. */
int rss_server_stats_get(rss_server_t s, rss_server_stats* out);
/* rss_server_destroy -- finish queued work, stop the workers, free everything. */
int rss_server_destroy(rss_server_t s);

/* rss_last_error -- message for the last failure on this thread ("" if none). */
const char* rss_last_error(void);

/* rss_error_string -- static name of a status code. */
const char* rss_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* RSS_H */
