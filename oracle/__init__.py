"""CPU FP64 oracle for strong recursive skeletonization (RS-S).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never does,
and the two share no code.

Written from the paper (Liang, Chen, Martinsson, Biros, "An O(N)
distributed-memory parallel direct solver for planar integral equations"):

* kernels.py      -- matrix entries (Sec. 1 eqs. e:axb/e:aij, Sec. 5 eqs.
                     e:kernel_laplace, e:kernel_helmholtz, e:a1, e:b1)
* tree.py         -- perfect quadtree, neighbour lists N(B), distance-2 lists
                     M(B) (Sec. 2.1, Def. d:m), box colours
* cpqr.py         -- interpolative decomposition by column-pivoted QR
                     (Sec. 2.2 Def. 1, Sec. 2.3 eqs. e:con/e:t)
* rss.py          -- the factorization (Sec. 2.4 eqs. e:s, e:step, e:sk;
                     Sec. 2.5 eqs. e:level, e:alg, Alg. a:fact) and the solve
                     (Sec. 2.6)
* dense_literal.py-- the same factorization applied literally to the full
                     N x N matrix (a bookkeeping check)
* matvec.py       -- exact products A x (dense, and BTTB-FFT on grids, as the
                     paper does in Sec. 5) and iterative refinement

Every function names the passage it follows.  Precision is FP64 / complex128
throughout.  Every function is pinned by a CPU test against something other
than itself (closed forms, library routines on special cases, brute force on
tiny inputs, exactness on degenerate kernels); functions without such a pin say
"parity unpinned" in their docstring.
"""
